// SOGRAND component decoding and block-turbo product decoding on gfx950.
//
// One 64-lane wavefront decodes one component word:
//   1. hard decision y, its syndrome s0 = XOR of the H columns where y = 1 and
//      its parity (section "Background on GRAND": H c = 0; even-code parity);
//   2. reliability ranks: a bitonic sort of (|lambda|, index) across lanes;
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
#include <cmath>

#include "internal.hpp"

namespace sg {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

struct WaveLds {
    double rho_r[SOGRAND_NMAX + 1];      // rho by rank (1..n); [0] = 1 for zero padding
    uint64_t key_b[SOGRAND_NMAX + 2];    // |lambda| bit patterns by bit index, padded with ~0
    double tau_l[SOGRAND_LIST_MAX];      // prod rho of each found pattern
    uint4 pat_l[SOGRAND_LIST_MAX];       // found patterns (ranks)
    uint32_t hs_r[SOGRAND_NMAX + 1];     // H column by rank; [0] = 0
    uint32_t q_l[SOGRAND_LIST_MAX];      // query number of each found codeword
    uint8_t pi_r[SOGRAND_NMAX + 1];      // bit index of each rank
    uint8_t zf[SOGRAND_NMAX];            // membership flags of one found pattern, by bit index
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
        return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false);
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

// parity-class masses of two disjoint bit sets combined (see decode_word step 3)
template <int M>
__device__ __forceinline__ void eo_combine(double &E, double &O) {
    const double E2 = xor_lane_f64<M>(E), O2 = xor_lane_f64<M>(O);
    const double nE = (E + E2) + (E * E2 + O * O2);
    const double nO = (O + O2) + (E * O2 + O * E2);
    E = nE;
    O = nO;
}

// One rank of a pattern: r is byte SH/8 of dword d.
#define SG_RANK(d, SH)                                   \
    do {                                                 \
        const uint32_t r_ = ((d) >> (SH)) & 0xffu;       \
        s ^= S.hs_r[r_];                                 \
        tau *= S.rho_r[r_];                              \
    } while (0)

// Decodes one word held as lam[slot] at bit index lane + 64*slot (< n).
// Writes the APP LLRs of the lane's bits into lapp; the list is left in S.
template <int NS>
__device__ __forceinline__ WordStats decode_word(const DevCode &c, int L, uint32_t qcap,
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
        rho[b] = valid[b] ? exp(-a) : 0.0;
        if (i < SOGRAND_NMAX + 2) S.key_b[i] = key[b];
    }
    if (NB == 1 && lane < 2) S.key_b[kWave + lane] = ~0ull;
    const uint32_t s0 = wave_xor(spart);
    const int par = ycount & 1;
    wave_sync();

    // 2. reliability rank of each bit: the number of smaller keys (bit patterns of
    //    non-negative doubles order like the values), ties broken by the bit index
    uint32_t cnt[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) cnt[b] = 0;
    for (int j = 0; j < n; j += 2) {
        const uint64_t k0 = S.key_b[j], k1 = S.key_b[j + 1];
#pragma unroll
        for (int b = 0; b < NB; b++) {
            cnt[b] += (k0 < key[b]) ? 1u : 0u;
            cnt[b] += (k1 < key[b]) ? 1u : 0u;
        }
    }
    {
        uint32_t part = 0;
#pragma unroll
        for (int b = 0; b < NB; b++) part += valid[b] ? cnt[b] : 0u;
        const uint32_t tot = __builtin_amdgcn_readfirstlane(wave_add(part));
        if (tot != (uint32_t)(n * (n - 1) / 2)) {
            // equal keys share a count: order each group of equal keys by bit index
            for (int j = 0; j < n; j++) {
                const uint64_t kj = S.key_b[j];
#pragma unroll
                for (int b = 0; b < NB; b++) cnt[b] += (kj == key[b] && j < lane + kWave * b) ? 1u : 0u;
            }
        }
    }
    int myrank[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        myrank[b] = valid[b] ? (int)cnt[b] + 1 : 0;
        if (valid[b]) {
            S.hs_r[myrank[b]] = c.hcol[i];
            S.rho_r[myrank[b]] = rho[b];
            S.pi_r[myrank[b]] = (uint8_t)i;
        }
    }
    if (lane == 0) {
        S.hs_r[0] = 0u;
        S.rho_r[0] = 1.0;
    }

    // 3. parity-class masses: adding bit i maps (E, O) to (E + O rho_i, O + (1 + E) rho_i);
    //    two disjoint bit sets combine as E = E1 + E2 + E1 E2 + O1 O2, O = O1 + O2 + E1 O2 + O1 E2
    double E = 0.0, O = 0.0;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        if (valid[b]) {
            const double e2 = E + O * rho[b];
            const double o2 = O + (1.0 + E) * rho[b];
            E = e2;
            O = o2;
        }
    }
    eo_combine<1>(E, O);
    eo_combine<2>(E, O);
    eo_combine<4>(E, O);
    eo_combine<8>(E, O);
    eo_combine<16>(E, O);
    eo_combine<32>(E, O);
    E = bcast0(E);
    O = bcast0(O);
    wave_sync();

    // 4. query loop over the schedule of the word's parity class; the next chunk's
    //    patterns are fetched while the current one is tested
    const int cls = c.even ? par : 0;
    const uint4 *__restrict__ tab = c.pat[cls];
    const uint32_t *__restrict__ wm = c.wmax[cls];
    const uint32_t limit = qcap < c.len[cls] ? qcap : c.len[cls];
    int found = 0;
    uint32_t Q = 0;
    double s_lane = 0.0;   // this lane's share of the tested nonzero-pattern mass (relative to p(0|r))
    uint32_t w_lane = 0;   // this lane's share of the tested pattern weights (counting only)
    uint4 e_next = make_uint4(0u, 0u, 0u, 0u);
    if ((uint32_t)lane < limit) e_next = tab[lane];
    uint32_t wm_next = wm[0];
    for (uint32_t base = 0; base < limit; base += kWave) {
        const uint4 e = e_next;
        const uint32_t wmx = wm_next;
        const uint32_t nb = base + kWave;
        if (nb < limit) {
            e_next = make_uint4(0u, 0u, 0u, 0u);
            if (nb + (uint32_t)lane < limit) e_next = tab[nb + lane];
            wm_next = wm[nb >> 6];
        }
        const bool act = base + (uint32_t)lane < limit;
        uint32_t s = s0;
        double tau = 1.0;
        if (wmx > 0) SG_RANK(e.x, 0);
        if (wmx > 1) SG_RANK(e.x, 8);
        if (wmx > 2) SG_RANK(e.x, 16);
        if (wmx > 3) SG_RANK(e.x, 24);
        if (wmx > 4) {
            SG_RANK(e.y, 0);
            if (wmx > 5) SG_RANK(e.y, 8);
            if (wmx > 6) SG_RANK(e.y, 16);
            if (wmx > 7) SG_RANK(e.y, 24);
            if (wmx > 8) {
                SG_RANK(e.z, 0);
                if (wmx > 9) SG_RANK(e.z, 8);
                if (wmx > 10) SG_RANK(e.z, 16);
                if (wmx > 11) SG_RANK(e.z, 24);
                if (wmx > 12) {
                    SG_RANK(e.w, 0);
                    if (wmx > 13) SG_RANK(e.w, 8);
                    if (wmx > 14) SG_RANK(e.w, 16);
                    if (wmx > 15) SG_RANK(e.w, 24);
                }
            }
        }
        uint64_t m = __ballot(act && s == 0u);
        int cut = kWave - 1;
        while (m != 0ull && found < L) {
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
        }
        const bool nonzero = (e.x & 0xffu) != 0u;
        if (act && nonzero && lane <= cut) s_lane += tau;
        if (count && act && lane <= cut) w_lane += pattern_weight(e);
        if (found >= L) {
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
        const double qs = 1.0 / (1.0 + rho[b]);   // p(bit = y | soft input)
        const double qf = rho[b] * qs;            // p(bit != y | soft input)
        N0[b] = pnf * (ybit[b] ? qf : qs);
        N1[b] = pnf * (ybit[b] ? qs : qf);
    }
    if (!degenerate) {
        const double invD = 1.0 / D;
        for (int l = 0; l < found; l++) {
            // membership flags of pattern l: clear, then mark the bits of its ranks
#pragma unroll
            for (int b = 0; b < NB; b++)
                if (lane + kWave * b < SOGRAND_NMAX) S.zf[lane + kWave * b] = 0;
            wave_sync();
            const uint4 pl = S.pat_l[l];
            if (lane < 16) {
                const uint32_t d = lane < 4 ? pl.x : (lane < 8 ? pl.y : (lane < 12 ? pl.z : pl.w));
                const uint32_t r = (d >> (8 * (lane & 3))) & 0xffu;
                if (r) S.zf[S.pi_r[r]] = 1;
            }
            wave_sync();
            const double P = S.tau_l[l] * invD;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const int i = lane + kWave * b;
                const int z = i < SOGRAND_NMAX ? S.zf[i] : 0;
                if (ybit[b] ^ z) N1[b] += P;
                else N0[b] += P;
            }
            wave_sync();
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        double la = log(N0[b] / N1[b]);
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
    if (count) st.ranks = wave_add(w_lane);
    return st;
}

// ----------------------------------------------------------------------------
// component decoding
// ----------------------------------------------------------------------------
struct ComponentArgs {
    DevCode code;
    int L;
    uint32_t qcap;
    size_t nwords;
    const void *llr_in;
    void *llr_app;
    void *llr_ext;
    uint8_t *hard;
    uint32_t *n_queries;
    uint8_t *n_found;
    uint32_t *found_q;
    double *p_found;
    double *p_notfound;
    uint8_t *found_z;
    ProfCounters *prof;
};

__device__ __forceinline__ void prof_add(ProfCounters *p, const WordStats &st) {
    atomicAdd(&p->words, 1ull);
    atomicAdd(&p->queries, (unsigned long long)st.Q);
    atomicAdd(&p->ranks, (unsigned long long)st.ranks);
}

template <typename T, int NS>
__global__ __launch_bounds__(kBlock) void k_component(ComponentArgs a) {
    constexpr int NB = Lanes<NS>::NB;
    __shared__ WaveLds lds[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const size_t wid = (size_t)blockIdx.x * kWavesPerBlock + wave;
    if (wid >= a.nwords) return;
    WaveLds &S = lds[wave];
    const int n = a.code.n;
    const T *in = static_cast<const T *>(a.llr_in) + wid * n;
    double lam[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        lam[b] = i < n ? (double)in[i] : 0.0;
    }
    double lapp[NB];
    const WordStats st = decode_word<NS>(a.code, a.L, a.qcap, lam, S, lapp, lane, a.prof != nullptr);
    if (a.prof && lane == 0) prof_add(a.prof, st);
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        if (i >= n) continue;
        const size_t o = wid * n + i;
        if (a.llr_app) static_cast<T *>(a.llr_app)[o] = (T)lapp[b];
        if (a.llr_ext) static_cast<T *>(a.llr_ext)[o] = (T)(lapp[b] - lam[b]);
        if (a.hard) a.hard[o] = lapp[b] < 0.0;
    }
    if (lane == 0) {
        if (a.n_queries) a.n_queries[wid] = st.Q;
        if (a.n_found) a.n_found[wid] = (uint8_t)st.found;
        if (a.p_notfound) a.p_notfound[wid] = st.pnf;
    }
    if (lane < a.L) {
        const bool f = lane < st.found;
        if (a.found_q) a.found_q[wid * a.L + lane] = f ? S.q_l[lane] : 0u;
        if (a.p_found) a.p_found[wid * a.L + lane] = f ? S.tau_l[lane] / st.D : 0.0;
    }
    if (a.found_z) {
        for (int l = 0; l < a.L; l++) {
            if (l < st.found) {
#pragma unroll
                for (int b = 0; b < NB; b++)
                    if (lane + kWave * b < SOGRAND_NMAX) S.zf[lane + kWave * b] = 0;
                wave_sync();
                const uint4 pl = S.pat_l[l];
                if (lane < 16) {
                    const uint32_t d = lane < 4 ? pl.x : (lane < 8 ? pl.y : (lane < 12 ? pl.z : pl.w));
                    const uint32_t r = (d >> (8 * (lane & 3))) & 0xffu;
                    if (r) S.zf[S.pi_r[r]] = 1;
                }
                wave_sync();
            }
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const int i = lane + kWave * b;
                if (i >= n) continue;
                const uint8_t z = l < st.found ? S.zf[i] : 0;
                a.found_z[(wid * a.L + l) * n + i] = z;
            }
            wave_sync();
        }
    }
}

// ----------------------------------------------------------------------------
// product codes
// ----------------------------------------------------------------------------
struct ProductArgs {
    DevCode code;
    int L;
    uint32_t qcap;
    double alpha;
    size_t nframes;
    const void *llr_ch;     // [F][n][n]
    void *la;               // [F][n][n] a-priori LLRs (work buffer)
    void *llr_app;          // [F][n][n] or NULL
    uint8_t *hard;          // [F][n][n]
    uint64_t *masks;        // [F][n][2] hard decision of each line of the last pass
    uint32_t *done;         // [F]
    uint32_t *halfmax;      // [F] largest query count of the current half-iteration
    uint64_t *sumq;         // [F]
    uint64_t *summax;       // [F]
    uint8_t *success;       // [F]
    uint16_t *half_iters;   // [F]
    int early_stop;
    ProfCounters *prof;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_product_init(ProductArgs a) {
    const int n = a.code.n;
    const size_t total = a.nframes * (size_t)n * n;
    T *la = static_cast<T *>(a.la);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        la[i] = (T)0;
    for (size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x; f < a.nframes; f += (size_t)gridDim.x * blockDim.x) {
        a.done[f] = 0u;
        a.halfmax[f] = 0u;
        a.sumq[f] = 0ull;
        a.summax[f] = 0ull;
        a.success[f] = 0;
        a.half_iters[f] = 0;
    }
}

// One wave per line: ROWS decodes row `line` of L_Ch + L_A, otherwise column `line`.
template <typename T, int NS, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_product_pass(ProductArgs a) {
    constexpr int NB = Lanes<NS>::NB;
    __shared__ WaveLds lds[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int n = a.code.n;
    const size_t wid = (size_t)blockIdx.x * kWavesPerBlock + wave;
    const size_t f = wid / n;
    const int line = (int)(wid % n);
    if (f >= a.nframes) return;
    if (a.done[f]) return;
    WaveLds &S = lds[wave];
    const T *ch = static_cast<const T *>(a.llr_ch) + f * n * n;
    T *la = static_cast<T *>(a.la) + f * n * n;
    double lam[NB];
    int pos[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        pos[b] = ROWS ? line * n + i : i * n + line;
        lam[b] = i < n ? (double)ch[pos[b]] + (double)la[pos[b]] : 0.0;
    }
    double lapp[NB];
    const WordStats st = decode_word<NS>(a.code, a.L, a.qcap, lam, S, lapp, lane, a.prof != nullptr);
    if (a.prof && lane == 0) prof_add(a.prof, st);
    uint64_t hm[2] = {0ull, 0ull};
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        const bool v = i < n;
        const bool neg = v && lapp[b] < 0.0;
        hm[b] = __ballot(neg);
        if (!v) continue;
        const double le = lapp[b] - lam[b];
        la[pos[b]] = (T)(a.alpha * le);
        if (a.llr_app) static_cast<T *>(a.llr_app)[f * n * n + pos[b]] = (T)lapp[b];
        a.hard[f * n * n + pos[b]] = neg;
    }
    if (lane == 0) {
        a.masks[(f * n + line) * 2 + 0] = hm[0];
        a.masks[(f * n + line) * 2 + 1] = hm[1];
        atomicAdd(reinterpret_cast<unsigned long long *>(&a.sumq[f]), (unsigned long long)st.Q);
        atomicMax(&a.halfmax[f], st.Q);
    }
}

// One wave per frame after half-iteration h: every line of the last pass and every
// cross line must have a zero syndrome.
__global__ __launch_bounds__(kBlock) void k_product_check(ProductArgs a, int h, int last) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const size_t f = (size_t)blockIdx.x * kWavesPerBlock + wave;
    if (f >= a.nframes) return;
    if (a.done[f]) return;
    const int n = a.code.n;
    const uint64_t *mk = a.masks + f * n * 2;
    bool bad = false;
    for (int b = 0; b < 2; b++) {
        const int x = lane + kWave * b;
        if (x >= n) continue;
        // x as a line of the last pass: XOR of the columns of its set bits
        const uint64_t m0 = mk[x * 2], m1 = mk[x * 2 + 1];
        uint32_t s = 0;
        for (int i = 0; i < n; i++) {
            const uint64_t bit = i < 64 ? (m0 >> i) & 1ull : (m1 >> (i - 64)) & 1ull;
            if (bit) s ^= a.code.hcol[i];
        }
        // x as a cross line: bit x of every line
        uint32_t t = 0;
        for (int l = 0; l < n; l++) {
            const uint64_t w = x < 64 ? mk[l * 2] : mk[l * 2 + 1];
            if ((w >> (x & 63)) & 1ull) t ^= a.code.hcol[l];
        }
        bad |= (s != 0u) || (t != 0u);
    }
    const bool valid = __ballot(bad) == 0ull;
    if (lane == 0) {
        a.summax[f] += a.halfmax[f];
        a.halfmax[f] = 0u;
        if ((valid && a.early_stop) || last) {
            a.done[f] = 1u;
            a.success[f] = valid;
            a.half_iters[f] = (uint16_t)h;
        }
    }
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------
static int sort_width(int n) { return n <= 32 ? 32 : (n <= 64 ? 64 : 128); }

template <typename T>
static void launch_component(const ComponentArgs &a, int ns, dim3 g, hipStream_t st) {
    if (ns == 32) hipLaunchKernelGGL((k_component<T, 32>), g, dim3(kBlock), 0, st, a);
    else if (ns == 64) hipLaunchKernelGGL((k_component<T, 64>), g, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_component<T, 128>), g, dim3(kBlock), 0, st, a);
}

template <typename T, bool ROWS>
static void launch_pass(const ProductArgs &a, int ns, dim3 g, hipStream_t st) {
    if (ns == 32) hipLaunchKernelGGL((k_product_pass<T, 32, ROWS>), g, dim3(kBlock), 0, st, a);
    else if (ns == 64) hipLaunchKernelGGL((k_product_pass<T, 64, ROWS>), g, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_product_pass<T, 128, ROWS>), g, dim3(kBlock), 0, st, a);
}

}  // namespace sg

extern "C" {

int sogrand_decode_component(const sogrand_code_t *code, const sogrand_params_t *params, size_t nwords,
                             const void *llr_in, void *llr_app, void *llr_ext, uint8_t *hard,
                             uint32_t *n_queries, uint8_t *n_found, uint32_t *found_q, double *p_found,
                             double *p_notfound, uint8_t *found_z, void *stream) {
    using namespace sg;
    SG_TRY(check_params(params));
    if (!code) return fail(SOGRAND_EINVAL, "code is NULL");
    if (nwords == 0) return SOGRAND_OK;
    if (!llr_in) return fail(SOGRAND_EINVAL, "llr_in is NULL");
    if (nwords > ((size_t)1 << 40) / (size_t)code->n) return fail(SOGRAND_EINVAL, "nwords too large");
    ComponentArgs a;
    SG_TRY(prepare_code(const_cast<sogrand_code_t *>(code), params->query_cap, &a.code));
    a.L = params->list_max;
    a.qcap = params->query_cap;
    a.nwords = nwords;
    a.llr_in = llr_in;
    a.llr_app = llr_app;
    a.llr_ext = llr_ext;
    a.hard = hard;
    a.n_queries = n_queries;
    a.n_found = n_found;
    a.found_q = found_q;
    a.p_found = p_found;
    a.p_notfound = p_notfound;
    a.found_z = found_z;
    a.prof = prof_counters(PK_COMPONENT);
    const size_t blocks = (nwords + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffffull) return fail(SOGRAND_EINVAL, "nwords too large for one launch");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int ns = sort_width(code->n);
    const int tok = prof_start(PK_COMPONENT, st);
    if (params->precision == SOGRAND_F64) launch_component<double>(a, ns, dim3((unsigned)blocks), st);
    else launch_component<float>(a, ns, dim3((unsigned)blocks), st);
    prof_stop(tok, st);
    SG_HIP(hipGetLastError());
    return SOGRAND_OK;
}

int sogrand_decode_product(const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes,
                           const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                           uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                           void *stream) {
    using namespace sg;
    SG_TRY(check_params(params));
    if (!code) return fail(SOGRAND_EINVAL, "code is NULL");
    if (nframes == 0) return SOGRAND_OK;
    if (!llr_ch || !hard || !success) return fail(SOGRAND_EINVAL, "llr_ch, hard and success are required");
    const int n = code->n;
    const size_t words = nframes * (size_t)n;
    if (nframes > ((size_t)1 << 34) / ((size_t)n * n)) return fail(SOGRAND_EINVAL, "nframes too large");
    const size_t blocks = (words + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffffull) return fail(SOGRAND_EINVAL, "nframes too large for one launch");
    ProductArgs a;
    SG_TRY(prepare_code(const_cast<sogrand_code_t *>(code), params->query_cap, &a.code));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t esz = params->precision == SOGRAND_F64 ? sizeof(double) : sizeof(float);
    // work buffer layout: la | masks | done | halfmax | sumq | summax | half_iters
    const size_t off_la = 0;
    const size_t off_mk = (off_la + nframes * n * n * esz + 255) & ~(size_t)255;
    const size_t off_dn = (off_mk + nframes * n * 2 * sizeof(uint64_t) + 255) & ~(size_t)255;
    const size_t off_hm = (off_dn + nframes * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t off_sq = (off_hm + nframes * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t off_sm = (off_sq + nframes * sizeof(uint64_t) + 255) & ~(size_t)255;
    const size_t off_hi = (off_sm + nframes * sizeof(uint64_t) + 255) & ~(size_t)255;
    const size_t total = off_hi + nframes * sizeof(uint16_t);
    char *ws = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&ws), total, st) != hipSuccess)
        return fail(SOGRAND_ENOMEM, "work buffer allocation of %zu bytes failed", total);
    a.L = params->list_max;
    a.qcap = params->query_cap;
    a.alpha = params->alpha;
    a.nframes = nframes;
    a.llr_ch = llr_ch;
    a.la = ws + off_la;
    a.llr_app = llr_app;
    a.hard = hard;
    a.masks = reinterpret_cast<uint64_t *>(ws + off_mk);
    a.done = reinterpret_cast<uint32_t *>(ws + off_dn);
    a.halfmax = reinterpret_cast<uint32_t *>(ws + off_hm);
    a.sumq = sum_queries ? sum_queries : reinterpret_cast<uint64_t *>(ws + off_sq);
    a.summax = sum_max_queries ? sum_max_queries : reinterpret_cast<uint64_t *>(ws + off_sm);
    a.success = success;
    a.half_iters = half_iters ? half_iters : reinterpret_cast<uint16_t *>(ws + off_hi);
    a.early_stop = params->early_stop ? 1 : 0;
    a.prof = prof_counters(PK_PASS);
    const int ns = sort_width(n);
    const bool f64 = params->precision == SOGRAND_F64;
    int rc = SOGRAND_OK;
    {
        const size_t ib = (nframes * n * n + kBlock - 1) / kBlock;
        const unsigned ig = (unsigned)(ib < 65536 ? ib : 65536);
        int tok = prof_start(PK_INIT, st);
        if (f64) hipLaunchKernelGGL(k_product_init<double>, dim3(ig), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL(k_product_init<float>, dim3(ig), dim3(kBlock), 0, st, a);
        prof_stop(tok, st);
        const unsigned cg = (unsigned)((nframes + kWavesPerBlock - 1) / kWavesPerBlock);
        for (int h = 1; h <= 2 * params->max_iter; h++) {
            const bool rows = (h & 1) != 0;
            tok = prof_start(PK_PASS, st);
            if (f64) {
                if (rows) launch_pass<double, true>(a, ns, dim3((unsigned)blocks), st);
                else launch_pass<double, false>(a, ns, dim3((unsigned)blocks), st);
            } else {
                if (rows) launch_pass<float, true>(a, ns, dim3((unsigned)blocks), st);
                else launch_pass<float, false>(a, ns, dim3((unsigned)blocks), st);
            }
            prof_stop(tok, st);
            tok = prof_start(PK_CHECK, st);
            hipLaunchKernelGGL(k_product_check, dim3(cg), dim3(kBlock), 0, st, a, h, h == 2 * params->max_iter ? 1 : 0);
            prof_stop(tok, st);
        }
        if (hipGetLastError() != hipSuccess) rc = fail(SOGRAND_EDEVICE, "product kernel launch failed");
    }
    (void)hipFreeAsync(ws, st);
    return rc;
}

}  // extern "C"
