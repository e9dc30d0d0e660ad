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
    double rho_r[SOGRAND_NMAX + 1];      // by rank (1..n); [0] = 1 for zero padding
    double rho_b[SOGRAND_NMAX];          // by bit index
    double tau_l[SOGRAND_LIST_MAX];      // prod rho of each found pattern
    uint64_t z_l[SOGRAND_LIST_MAX][2];   // found patterns as bit masks over bit indices
    uint32_t hs_r[SOGRAND_NMAX + 1];     // H column by rank; [0] = 0
    uint32_t q_l[SOGRAND_LIST_MAX];      // query number of each found codeword
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
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v ^= __shfl_xor(v, d);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d);
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

__device__ __forceinline__ bool key_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// Bitonic sort of NS (key, index) pairs; element e = lane + 64*slot.  Keys are the
// bit patterns of |lambda| (monotone for non-negative doubles); ties fall back to
// the bit index.  Afterwards element e holds rank e+1.
template <int NS>
__device__ __forceinline__ void bitonic_sort(uint64_t (&key)[Lanes<NS>::NB], uint32_t (&idx)[Lanes<NS>::NB], int lane) {
    constexpr int NB = Lanes<NS>::NB;
#pragma unroll
    for (int k = 2; k <= NS; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= kWave) {
                // NS = 128, j = 64: the partner is the same lane's other slot; k = 128 sorts up
                if constexpr (NB > 1) {
                    if (key_less(key[NB - 1], idx[NB - 1], key[0], idx[0])) {
                        uint64_t tk = key[0]; key[0] = key[NB - 1]; key[NB - 1] = tk;
                        uint32_t ti = idx[0]; idx[0] = idx[NB - 1]; idx[NB - 1] = ti;
                    }
                }
            } else {
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    const int e = lane + kWave * b;
                    const uint64_t ok = __shfl_xor(key[b], j);
                    const uint32_t oi = __shfl_xor(idx[b], j);
                    const bool lower = (e & j) == 0;
                    const bool up = (e & k) == 0;
                    const bool other_less = key_less(ok, oi, key[b], idx[b]);
                    // the lower element of an ascending pair keeps the minimum
                    const bool take = (lower == up) ? other_less : !other_less;
                    if (take) { key[b] = ok; idx[b] = oi; }
                }
            }
        }
    }
}

// Decodes one word held as lam[slot] at bit index lane + 64*slot (< n).
// Writes the APP LLRs of the lane's bits into lapp; the list is left in S.
template <int NS>
__device__ __forceinline__ WordStats decode_word(const DevCode &c, int L, uint32_t qcap,
                                                 const double (&lam)[Lanes<NS>::NB], WaveLds &S,
                                                 double (&lapp)[Lanes<NS>::NB], int lane) {
    constexpr int NB = Lanes<NS>::NB;
    const int n = c.n;

    // 1. hard decision, syndrome and parity
    bool valid[NB];
    int ybit[NB];
    uint32_t spart = 0;
    int ycount = 0;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        valid[b] = i < n;
        ybit[b] = valid[b] && lam[b] < 0.0;
        if (ybit[b]) spart ^= c.hcol[i];
        ycount += __popcll(__ballot(ybit[b]));
    }
    const uint32_t s0 = wave_xor(spart);
    const int par = ycount & 1;

    // 2. rho by bit index, then the reliability sort
    double rho[NB];
    uint64_t key[NB];
    uint32_t idx[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        const double a = fabs(lam[b]);
        rho[b] = valid[b] ? exp(-a) : 0.0;
        if (valid[b]) S.rho_b[i] = rho[b];
        key[b] = valid[b] ? (uint64_t)__double_as_longlong(a) : ~0ull;
        idx[b] = (uint32_t)i;
    }
    bitonic_sort<NS>(key, idx, lane);
    wave_sync();
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int e = lane + kWave * b;
        if (e < n) {
            const int r = e + 1;
            S.hs_r[r] = c.hcol[idx[b]];
            S.rho_r[r] = S.rho_b[idx[b]];
            S.rank_b[idx[b]] = (uint8_t)r;
        }
    }
    if (lane == 0) {
        S.hs_r[0] = 0u;
        S.rho_r[0] = 1.0;
    }
    wave_sync();
    int myrank[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) myrank[b] = valid[b] ? S.rank_b[lane + kWave * b] : 0;

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
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double E2 = __shfl_xor(E, d), O2 = __shfl_xor(O, d);
        const double nE = (E + E2) + (E * E2 + O * O2);
        const double nO = (O + O2) + (E * O2 + O * E2);
        E = nE;
        O = nO;
    }
    E = bcast0(E);
    O = bcast0(O);

    // 4. query loop over the schedule of the word's parity class
    const int cls = c.even ? par : 0;
    const uint4 *__restrict__ tab = c.pat[cls];
    const uint8_t *__restrict__ wm = c.wmax[cls];
    const uint32_t limit = qcap < c.len[cls] ? qcap : c.len[cls];
    int found = 0;
    uint32_t Q = 0;
    double s_lane = 0.0;   // this lane's share of the tested nonzero-pattern mass (relative to p(0|r))
    for (uint32_t base = 0; base < limit; base += kWave) {
        const uint32_t g = base + (uint32_t)lane;
        const bool act = g < limit;
        uint4 e = make_uint4(0u, 0u, 0u, 0u);
        if (act) e = tab[g];
        const int wmx = wm[base >> 6];
        const uint32_t wd[4] = {e.x, e.y, e.z, e.w};
        uint32_t s = s0;
        double tau = 1.0;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            if (j >= wmx) break;
            const uint32_t r = (wd[j >> 2] >> (8 * (j & 3))) & 0xffu;
            s ^= S.hs_r[r];
            tau *= S.rho_r[r];
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
            const uint32_t hd[4] = {hx, hy, hz, hw};
            uint64_t zm[NB];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                bool in = false;
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    if (j >= wmx) break;
                    const int r = (int)((hd[j >> 2] >> (8 * (j & 3))) & 0xffu);
                    in |= (r != 0) && (r == myrank[b]);
                }
                zm[b] = __ballot(in);
            }
            if (lane == 0) {
                S.tau_l[found] = th;
                S.q_l[found] = base + (uint32_t)h + 1u;
                S.z_l[found][0] = zm[0];
                S.z_l[found][1] = NB > 1 ? zm[NB - 1] : 0ull;
            }
            found++;
            if (found == L) cut = h;
        }
        const bool nonzero = (e.x & 0xffu) != 0u;
        if (act && nonzero && lane <= cut) s_lane += tau;
        if (found >= L) {
            Q = base + (uint32_t)cut + 1u;
            break;
        }
        Q = limit < base + kWave ? limit : base + kWave;
    }
    wave_sync();
    const double Snz = bcast0(wave_sum(s_lane));

    // 5. Corollary 1 inside the parity class: not-found mass M = (class mass) - (tested mass),
    //    both relative to p(0|r); the zero pattern (first in its class) cancels exactly.
    const double T = c.even ? (par ? O : E) : (E + O);
    double M = T - Snz;
    if (!(M > 0.0)) M = 0.0;
    double D = M * c.phi;
    for (int l = 0; l < found; l++) D += S.tau_l[l];
    double pnf = (M * c.phi) / D;
    const bool degenerate = !(D > 0.0) || !isfinite(D);
    if (degenerate) pnf = 1.0;   // every probability underflowed: keep the soft input

    // eq. (LLRi): list codewords weighted by their APPs, plus the soft input weighted by P_nf
#pragma unroll
    for (int b = 0; b < NB; b++) {
        double N0 = 0.0, N1 = 0.0;
        if (!degenerate) {
            for (int l = 0; l < found; l++) {
                const double P = S.tau_l[l] / D;
                const int z = (int)((S.z_l[l][b] >> lane) & 1ull);
                if (ybit[b] ^ z) N1 += P;
                else N0 += P;
            }
        }
        const double qs = 1.0 / (1.0 + rho[b]);   // p(bit = y | soft input)
        const double qf = rho[b] * qs;            // p(bit != y | soft input)
        if (ybit[b]) {
            N1 += pnf * qs;
            N0 += pnf * qf;
        } else {
            N0 += pnf * qs;
            N1 += pnf * qf;
        }
        double la = log(N0) - log(N1);
        if (!(la <= 1000.0)) la = 1000.0;
        if (!(la >= -1000.0)) la = -1000.0;
        lapp[b] = la;
    }
    WordStats st;
    st.Q = Q;
    st.found = found;
    st.pnf = pnf;
    st.D = D;
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
};

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
    const WordStats st = decode_word<NS>(a.code, a.L, a.qcap, lam, S, lapp, lane);
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
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const int i = lane + kWave * b;
                if (i >= n) continue;
                const uint8_t z = l < st.found ? (uint8_t)((S.z_l[l][b] >> lane) & 1ull) : 0;
                a.found_z[(wid * a.L + l) * n + i] = z;
            }
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
    const WordStats st = decode_word<NS>(a.code, a.L, a.qcap, lam, S, lapp, lane);
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
    const size_t blocks = (nwords + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffffull) return fail(SOGRAND_EINVAL, "nwords too large for one launch");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int ns = sort_width(code->n);
    if (params->precision == SOGRAND_F64) launch_component<double>(a, ns, dim3((unsigned)blocks), st);
    else launch_component<float>(a, ns, dim3((unsigned)blocks), st);
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
    const int ns = sort_width(n);
    const bool f64 = params->precision == SOGRAND_F64;
    int rc = SOGRAND_OK;
    {
        const size_t ib = (nframes * n * n + kBlock - 1) / kBlock;
        const unsigned ig = (unsigned)(ib < 65536 ? ib : 65536);
        if (f64) hipLaunchKernelGGL(k_product_init<double>, dim3(ig), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL(k_product_init<float>, dim3(ig), dim3(kBlock), 0, st, a);
        const unsigned cg = (unsigned)((nframes + kWavesPerBlock - 1) / kWavesPerBlock);
        for (int h = 1; h <= 2 * params->max_iter; h++) {
            const bool rows = (h & 1) != 0;
            if (f64) {
                if (rows) launch_pass<double, true>(a, ns, dim3((unsigned)blocks), st);
                else launch_pass<double, false>(a, ns, dim3((unsigned)blocks), st);
            } else {
                if (rows) launch_pass<float, true>(a, ns, dim3((unsigned)blocks), st);
                else launch_pass<float, false>(a, ns, dim3((unsigned)blocks), st);
            }
            hipLaunchKernelGGL(k_product_check, dim3(cg), dim3(kBlock), 0, st, a, h, h == 2 * params->max_iter ? 1 : 0);
        }
        if (hipGetLastError() != hipSuccess) rc = fail(SOGRAND_EDEVICE, "product kernel launch failed");
    }
    (void)hipFreeAsync(ws, st);
    return rc;
}

}  // extern "C"
