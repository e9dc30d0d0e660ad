// Two component words of up to 32 bits per wavefront: lanes 0-31 decode one word
// and lanes 32-63 another.  Each step is the one of decode_word (word.hpp), done
// over a half-wave: the reductions stop at a distance of 16 lanes, and every
// quantity that decode_word keeps wave-uniform is uniform per half instead.  The
// query loop tests 32 patterns of each word per round, so the two words advance
// through their own schedules side by side and the loop runs until both have
// stopped.  Results are those of decode_word on each word alone.
#pragma once

#include "word.hpp"

namespace sg {

// Scratch of one word of up to 32 bits (the fields of WaveLds, sized for 32 bits)
struct PairLds {
    uint4 ent_r[36];                     // by rank (1..32): rho (x, y), H column (z); [0]: rho 1, H 0
    uint64_t key_b[34];                  // |lambda| bit patterns by bit index, padded with ~0
    double tau_l[SOGRAND_LIST_MAX];      // prod rho of each found pattern
    uint4 pat_l[SOGRAND_LIST_MAX];       // found patterns (ranks)
    uint32_t q_l[SOGRAND_LIST_MAX];      // query number of each found codeword
    uint32_t zmask[32];                  // bit l set iff the bit lies in found pattern l
    uint8_t pi_r[33];                    // bit index of each rank
};

// Half-wave totals: the row prefix of the wave reductions (word.hpp) and the broadcast of
// lane 15 into rows 1 and 3 leave each half's total in its last lane (31, 63); every lane
// receives its own half's.
#define SG_HALF_REDUCE(IN, OP)                                                         \
    do {                                                                               \
        v = v OP IN<0x111, 0xF, true>(v);   /* row_shr:1 */                            \
        v = v OP IN<0x112, 0xF, true>(v);   /* row_shr:2 */                            \
        v = v OP IN<0x114, 0xF, true>(v);   /* row_shr:4 */                            \
        v = v OP IN<0x118, 0xF, true>(v);   /* row_shr:8 */                            \
        v = v OP IN<0x142, 0xA, false>(v);  /* row_bcast:15 into rows 1 and 3 */       \
    } while (0)

__device__ __forceinline__ uint32_t half_pick_u(uint32_t v, int lane, int l0) {
    const uint32_t a = __builtin_amdgcn_readlane(v, l0), b = __builtin_amdgcn_readlane(v, l0 + 32);
    return lane < 32 ? a : b;
}

__device__ __forceinline__ uint32_t half_xor(uint32_t v, int lane) {
    SG_HALF_REDUCE(dpp_in, ^);
    return half_pick_u(v, lane, 31);
}

__device__ __forceinline__ uint32_t half_add(uint32_t v, int lane) {
    SG_HALF_REDUCE(dpp_in, +);
    return half_pick_u(v, lane, 31);
}

__device__ __forceinline__ double half_sum(double v, int lane) {
    SG_HALF_REDUCE(dpp_in_f64, +);
    const double a = readlane_f64(v, 31), b = readlane_f64(v, 63);
    return lane < 32 ? a : b;
}

// inclusive prefix sum over the 32 lanes of a half, in lane order (Hillis-Steele)
__device__ __forceinline__ double half_scan_add(double v, int hl) {
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)u, d);
        const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(u >> 32), d);
        const double t = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
        if (hl >= d) v += t;
    }
    return v;
}

// zmask[bit] |= 1 << l for every bit of the half's found pattern l: lane hl handles
// byte hl % 16 of pattern hl / 16 (+ 2 per round)
__device__ __forceinline__ void mark_found_half(PairLds &S, int found, int hl) {
    for (int g = 0; g < found; g += 2) {
        const int l = g + (hl >> 4);
        if (l < found) {
            const uint4 pl = S.pat_l[l];
            const int j = hl & 15;
            const uint32_t d = j < 4 ? pl.x : (j < 8 ? pl.y : (j < 12 ? pl.z : pl.w));
            const uint32_t r = (d >> (8 * (j & 3))) & 0xffu;
            if (r) atomicOr(&S.zmask[S.pi_r[r]], 1u << l);
        }
    }
}

// Decodes the lane's word (bit lane % 32 held in lam; the word's scratch is S, one per
// half).  skip: this half holds no word (its lanes take part in the wave's steps, test
// no pattern and their outputs are meaningless).  Returns the word's statistics in
// every lane of its half and its APP LLR in lapp.  TABLE: the elementary functions
// read their coefficients through a pointer, as in decode_word (persistent kernels).
template <bool STOP, bool TABLE = false>
__device__ __forceinline__ WordStats decode_pair(const DevCode &c, int L, uint32_t qcap, double pstop, double lam,
                                                 bool skip, PairLds &S, double &lapp, int lane, bool count) {
    const int n = c.n;
    const int hl = lane & 31;
    const bool upper = lane >= 32;
    const bool valid = hl < n;

    // 1. hard decision, syndrome and parity; keys and rho
    const int ybit = valid && lam < 0.0;
    const uint64_t yb = __ballot(ybit);
    const int par = __popc(upper ? (uint32_t)(yb >> 32) : (uint32_t)yb) & 1;
    const uint32_t s0 = half_xor(ybit ? gptr(c.hcol)[hl] : 0u, lane);
    const double a = fabs(lam);
    const uint64_t key = valid ? (uint64_t)__double_as_longlong(a) : ~0ull;
    const double rho = valid ? exp_neg<TABLE>(a) : 0.0;

    // 2. ranks by counting smaller keys of the same word, ties by bit index
    S.key_b[hl] = key;
    if (hl < 2) S.key_b[32 + hl] = ~0ull;
    wave_sync();
    uint32_t cnt = 0;
    for (int j = 0; j < n; j += 2) {
        const uint64_t k0 = S.key_b[j], k1 = S.key_b[j + 1];
        cnt += (k0 < key) ? 1u : 0u;
        cnt += (k1 < key) ? 1u : 0u;
    }
    const uint32_t tot = half_add(valid ? cnt : 0u, lane);
    const bool exact_pass = tot != (uint32_t)(n * (n - 1) / 2);
    if (exact_pass) {
        for (int j = 0; j < n; j++) {
            const uint64_t kj = S.key_b[j];
            cnt += (kj == key && j < hl) ? 1u : 0u;
        }
    }
    const int myrank = valid ? (int)cnt + 1 : 0;
    if (valid) {
        S.ent_r[myrank].z = gptr(c.hcol)[hl];
        put_rho(S, myrank, rho);
        S.pi_r[myrank] = (uint8_t)hl;
    } else {
        put_rho(S, hl + 1, 0.0);   // ranks n+1 .. 32 carry rho = 0 for the unguarded fold
    }
    S.zmask[hl] = 0u;
    if (hl == 0) {
        S.ent_r[0].z = 0u;
        put_rho(S, 0, 1.0);
    }
    wave_sync();

    // 3. parity-class masses: lanes 0-3 of a half fold 8 ranks each, then combine
    const int grp = hl < 4 ? hl : 3;
    double E = 0.0, O = rho_at(S, 8 * grp + 1);
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
    {
        const double e0 = readlane_f64(E, 3), e1 = readlane_f64(E, 35);
        const double o0 = readlane_f64(O, 3), o1 = readlane_f64(O, 35);
        E = lane < 32 ? e0 : e1;
        O = lane < 32 ? o0 : o1;
    }

    // 4. query loop: each half tests 32 patterns of its word's class schedule per round
    const int cls = c.even ? par : 0;
    const auto *tab = gptr(cls ? c.pat[1] : c.pat[0]);
    const uint32_t len = cls ? c.len[1] : c.len[0];
    const uint32_t limit = skip ? 0u : (qcap < len ? qcap : len);
    const uint32_t lim0 = __builtin_amdgcn_readlane(limit, 0), lim1 = __builtin_amdgcn_readlane(limit, 32);
    const uint32_t lim_max = lim0 > lim1 ? lim0 : lim1;
    const int cls0 = __builtin_amdgcn_readlane(cls, 0), cls1 = __builtin_amdgcn_readlane(cls, 32);
    const auto *wm0 = gptr(cls0 ? c.wmax[1] : c.wmax[0]);
    const auto *wm1 = gptr(cls1 ? c.wmax[1] : c.wmax[0]);
    bool done = limit == 0u;
    bool stopped = false;
    int found = 0;
    uint32_t Q = 0;
    double s_lane = 0.0;
    uint32_t w_lane = 0;
    uint4 e_next = make_uint4(0u, 0u, 0u, 0u);
    if ((uint32_t)hl < limit) e_next = gload(tab, hl);
    for (uint32_t base = 0; base < lim_max; base += 32) {
        // both words have stopped
        if (__ballot(!done) == 0ull) break;
        const uint4 e = e_next;
        e_next = make_uint4(0u, 0u, 0u, 0u);
        if (!done && base + 32u + (uint32_t)hl < limit) e_next = gload(tab, base + 32u + hl);
        // largest pattern weight of the round over both words' 64-pattern chunks
        const uint32_t w0 = base < lim0 ? wm0[base >> 6] : 0u;
        const uint32_t w1 = base < lim1 ? wm1[base >> 6] : 0u;
        const uint32_t wmx = __builtin_amdgcn_readfirstlane(w0 > w1 ? w0 : w1);   // the same in every lane
        const bool act = !done && base + (uint32_t)hl < limit;
        uint32_t s = s0;
        double tau = 1.0;
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
        const bool hit = act && s == 0u;
        const uint64_t m = __ballot(hit);
        const uint32_t mh = upper ? (uint32_t)(m >> 32) : (uint32_t)m;   // this half's hits
        int cut = 31;
        // tested nonzero-pattern mass before this round, for the list-BLER stop
        double s_before = 0.0;
        if constexpr (STOP) {
            s_before = half_sum(s_lane, lane);
            const double tested = half_scan_add((act && (e.x & 0xffu) != 0u) ? tau : 0.0, hl);
            S.key_b[hl] = (uint64_t)__double_as_longlong(tested);
        }
        if (mh != 0u) {
            const int nh = __popc(mh);
            const uint32_t below = __popc(mh & ((1u << hl) - 1u));
            const uint32_t slot = (uint32_t)found + below;
            if (hit && slot < (uint32_t)L) {
                S.tau_l[slot] = tau;
                S.q_l[slot] = base + (uint32_t)hl + 1u;
                S.pat_l[slot] = e;
            }
            if constexpr (!STOP) {
                if (found + nh >= L) {
                    uint32_t mm = mh;
                    for (int k = found + 1; k < L; k++) mm &= mm - 1u;
                    cut = __builtin_ctz(mm);
                    found = L;
                } else {
                    found += nh;
                }
            }
        }
        if constexpr (STOP) {
            wave_sync();
            if (mh != 0u) {
                const double T = c.even ? (par ? O : E) : (E + O);
                uint32_t mm = mh;
                while (mm != 0u) {
                    const int h = __builtin_ctz(mm);
                    mm &= mm - 1u;
                    found++;
                    if (found == L) {
                        cut = h;
                        break;
                    }
                    double Mi = T - (s_before + __longlong_as_double((long long)S.key_b[h]));
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
            wave_sync();
        }
        const bool nonzero = (e.x & 0xffu) != 0u;
        if (act && nonzero && hl <= cut) s_lane += tau;
        if (count && act && hl <= cut) w_lane += pattern_weight(e);
        if (!done) {
            if (found >= L || stopped) {
                Q = base + (uint32_t)cut + 1u;
                done = true;
            } else {
                const uint32_t nb = base + 32u;
                Q = limit < nb ? limit : nb;
                done = nb >= limit;
            }
        }
    }

    const double Snz = half_sum(s_lane, lane);

    // 5. Corollary 1 inside the parity class (as decode_word)
    wave_sync();
    const double T = c.even ? (par ? O : E) : (E + O);
    double M = T - Snz;
    if (!(M > 0.0) || Q == class_size(c)) M = 0.0;
    double D = M * c.phi;
    for (int l = 0; l < found; l++) D += S.tau_l[l];
    const bool degenerate = !(D > 0.0) || !isfinite(D);
    const double invD = 1.0 / (degenerate ? 1.0 : D);
    const double pnf = degenerate ? 1.0 : (M * c.phi) * invD;

    // eq. (LLRi), both sums taken times 1 + rho (as decode_word)
    double N0 = 0.0, N1 = 0.0;
    if (!degenerate) mark_found_half(S, found, hl);
    wave_sync();
    if (!degenerate) {
        uint32_t zm = S.zmask[hl] ^ (ybit ? 0xffffffffu : 0u);
#pragma unroll 2
        for (int l = 0; l < found; l++) {
            const double P = S.tau_l[l] * invD;
            const double one = (double)((zm >> l) & 1u);
            N1 = fma(P, one, N1);
            N0 = fma(P, 1.0 - one, N0);
        }
    }
    const double opr = 1.0 + rho;
    const double sy = pnf, sf = pnf * rho;
    N0 = fma(opr, N0, ybit ? sf : sy);
    N1 = fma(opr, N1, ybit ? sy : sf);
    double la = log_ratio<TABLE>(N0, N1);
    if (!(la <= 1000.0)) la = 1000.0;
    if (!(la >= -1000.0)) la = -1000.0;
    lapp = la;

    WordStats st;
    st.Q = Q;
    st.found = found;
    st.pnf = pnf;
    st.D = D;
    st.ranks = 0;
    st.exact_rank = exact_pass ? 1 : 0;
#ifdef SG_PHASE_CLOCKS
    for (int q = 0; q < kPhases; q++) st.phase[q] = 0u;   // pairs are not timed by phase
#endif
    if (count) st.ranks = half_add(w_lane, lane);
    return st;
}

}  // namespace sg
