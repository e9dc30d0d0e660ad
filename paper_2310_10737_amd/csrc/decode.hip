// SOGRAND component decoding and plain block-turbo product decoding on gfx950:
// one launch per half-iteration plus a per-frame validity check.
#include <new>

#include "pair.hpp"

namespace sg {

// ----------------------------------------------------------------------------
// component decoding
// ----------------------------------------------------------------------------
struct ComponentArgs {
    DevCode code;
    int L;
    uint32_t qcap;
    double pstop;           // list-BLER stop threshold, 0 = off
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


template <typename T, int NS, int WPB, bool STOP>
__global__ __launch_bounds__(kWave * WPB) __attribute__((amdgpu_waves_per_eu(8))) void k_component(ComponentArgs a) {
    constexpr int NB = Lanes<NS>::NB;
    __shared__ WaveLds lds[WPB];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    WaveLds &S = lds[wave];
    const size_t wid = (size_t)blockIdx.x * WPB + wave;
    if (wid >= a.nwords) return;
    const int n = a.code.n;
    const T *in = static_cast<const T *>(a.llr_in) + wid * n;
    double lam[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        lam[b] = i < n ? (double)in[i] : 0.0;
    }
    double lapp[NB];
    const WordStats st = decode_word<NS, false, STOP>(a.code, nullptr, a.L, a.qcap, a.pstop, lam, S, lapp, lane,
                                                      a.prof != nullptr);
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
        // zmask was filled by the soft-output step unless every probability underflowed
        if (!(st.D > 0.0) || !isfinite(st.D)) mark_found(S, st.found, lane);
        for (int l = 0; l < a.L; l++) {
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const int i = lane + kWave * b;
                if (i >= n) continue;
                const uint8_t z = l < st.found ? (uint8_t)((S.zmask[i] >> l) & 1u) : 0;
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
    double pstop;           // list-BLER stop threshold, 0 = off
    double alpha;
    size_t nframes;
    const void *llr_ch;     // [F][n][n]
    // Work buffers, each [F][n][n], laid out so that every pass reads its lines
    // contiguously ("line-major": element i of line l at l * n + i): L_Ch in the
    // second family's line order (written by the first pass), the a-priori LLRs for
    // the first family's passes (written by the second family's passes) and for the
    // second family's passes (written by the first family's).  For a product code the
    // first family is the rows, so its line-major order is the frame's own.
    void *ch_t;
    void *la_rm;
    void *la_cm;
    void *ch_a;             // QC-GLDPC only: L_Ch in the first family's line order
    int first;              // this launch is the first row pass (no a-priori LLRs yet)
    int topo;               // kProduct or kGldpc
    void *llr_app;          // [F][n][n] or NULL
    uint8_t *hard;          // [F][n][n], written by the check kernel when the frame finishes
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

// Per-frame state at the start (the first row pass needs no a-priori LLRs and
// writes every element the column pass reads).
__global__ __launch_bounds__(kBlock) void k_product_init(ProductArgs a) {
    for (size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x; f < a.nframes; f += (size_t)gridDim.x * blockDim.x) {
        a.done[f] = 0u;
        a.halfmax[f] = 0u;
        a.sumq[f] = 0ull;
        a.summax[f] = 0ull;
        a.success[f] = 0;
        a.half_iters[f] = 0;
    }
}

// The two families of component words.  Product code: the rows (first family) and
// the columns.  QC-GLDPC (performance-evaluation section: adjacency matrix with block
// rows [I(0) ... I(0)] and [I(0) I(1) ... I(n-1)], I(i) the identity rotated right by
// i): variable node j*n + c is column c of block j; word `line` of the first block
// row takes its bit j from variable node j*n + line, of the second from
// j*n + (line + j) mod n.

template <int TOPO, bool FIRST_FAMILY>
struct Lines {
    // frame position (variable node) of bit i of word `line`
    static __device__ __forceinline__ uint32_t vn(uint32_t line, uint32_t i, uint32_t n) {
        if constexpr (TOPO == kProduct) return FIRST_FAMILY ? line * n + i : i * n + line;
        else return FIRST_FAMILY ? i * n + line : i * n + (line + i) % n;
    }
    // line-major position of the same variable node among the other family's words
    static __device__ __forceinline__ uint32_t cross(uint32_t line, uint32_t i, uint32_t n) {
        if constexpr (TOPO == kProduct) return i * n + line;
        else return (FIRST_FAMILY ? (line + n - i) % n : (line + i) % n) * n + i;
    }
};

// One wave per word: ROWS decodes word `line` of the first family (the rows of a
// product code) of L_Ch + L_A, otherwise of the second.
template <typename T, int NS, bool ROWS, int WPB, bool STOP, int TOPO>
__global__ __launch_bounds__(kWave * WPB) __attribute__((amdgpu_waves_per_eu(8))) void k_product_pass(ProductArgs a) {
    using LN = Lines<TOPO, ROWS>;
    constexpr int NB = Lanes<NS>::NB;
    __shared__ WaveLds lds[WPB];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    WaveLds &S = lds[wave];
    const uint32_t n = (uint32_t)a.code.n;
    // the host keeps nframes * n below 2^31
    const uint32_t wid = (uint32_t)blockIdx.x * WPB + (uint32_t)wave;
    const uint32_t f = wid / n;
    const uint32_t line = wid - f * n;
    if (f >= a.nframes) return;
    if (a.done[f]) return;
    const size_t fo = (size_t)f * n * n;   // element offset of frame f
    // inputs are read along the word (line-major); the a-priori LLRs for the other
    // family are written across.  A product code's rows read L_Ch from the frame
    // itself; a QC-GLDPC's first pass gathers it and keeps both line-major copies.
    const bool first = ROWS && a.first;
    const T *ch;
    if constexpr (TOPO == kProduct) ch = static_cast<const T *>(ROWS ? a.llr_ch : a.ch_t) + fo;
    else ch = static_cast<const T *>(ROWS ? a.ch_a : a.ch_t) + fo;
    const T *la_in = static_cast<const T *>(ROWS ? a.la_rm : a.la_cm) + fo;
    T *la_out = static_cast<T *>(ROWS ? a.la_cm : a.la_rm) + fo;
    double lam[NB];
    uint32_t pos[NB];   // frame position of the lane's bits
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const uint32_t i = (uint32_t)(lane + kWave * b);
        pos[b] = LN::vn(line, i, n);
        lam[b] = 0.0;
        if (i < n) {
            T c;
            if (TOPO == kGldpc && first) c = static_cast<const T *>(a.llr_ch)[fo + pos[b]];
            else c = ch[line * n + i];
            lam[b] = first ? (double)c : (double)c + (double)la_in[line * n + i];
            if (first) {
                static_cast<T *>(a.ch_t)[fo + LN::cross(line, i, n)] = c;
                if (TOPO == kGldpc) static_cast<T *>(a.ch_a)[fo + line * n + i] = c;
            }
        }
    }
    double lapp[NB];
    const WordStats st = decode_word<NS, false, STOP>(a.code, nullptr, a.L, a.qcap, a.pstop, lam, S, lapp, lane,
                                                      a.prof != nullptr);
    if (a.prof && lane == 0) prof_add(a.prof, st);
    uint64_t hm[2] = {0ull, 0ull};
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const uint32_t i = (uint32_t)(lane + kWave * b);
        const bool v = i < n;
        const bool neg = v && lapp[b] < 0.0;
        hm[b] = __ballot(neg);
        if (!v) continue;
        const double le = lapp[b] - lam[b];
        la_out[LN::cross(line, i, n)] = (T)(a.alpha * le);
        if (a.llr_app) static_cast<T *>(a.llr_app)[fo + pos[b]] = (T)lapp[b];
    }
    if (lane == 0) {
        a.masks[((size_t)f * n + line) * 2 + 0] = hm[0];
        a.masks[((size_t)f * n + line) * 2 + 1] = hm[1];
        atomicAdd(reinterpret_cast<unsigned long long *>(&a.sumq[f]), (unsigned long long)st.Q);
        atomicMax(&a.halfmax[f], st.Q);
    }
}

// Words of up to 32 bits, two per wave (decode_pair): lanes 0-31 take global word
// 2p and lanes 32-63 word 2p + 1 of pair p.  A half whose word lies past the last
// frame, or in a frame that has stopped, takes part without testing patterns.
template <typename T, bool ROWS, int WPB, bool STOP, int TOPO>
__global__ __launch_bounds__(kWave * WPB) void k_product_pass_pair(ProductArgs a) {
    using LN = Lines<TOPO, ROWS>;
    __shared__ PairLds lds[WPB][2];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const uint32_t hl = (uint32_t)(lane & 31);
    const bool upper = lane >= 32;
    PairLds &S = lds[wave][upper ? 1 : 0];
    const uint32_t n = (uint32_t)a.code.n;
    // the host keeps nframes * n below 2^31
    const uint32_t pair = (uint32_t)blockIdx.x * WPB + (uint32_t)wave;
    const uint32_t gl = pair * 2u + (upper ? 1u : 0u);
    const uint32_t f = gl / n;
    const uint32_t line = gl - f * n;
    const bool live = f < a.nframes && !a.done[f];
    if (__ballot(live) == 0ull) return;
    const size_t fo = (size_t)f * n * n;
    const bool first = ROWS && a.first;
    const T *ch;
    if constexpr (TOPO == kProduct) ch = static_cast<const T *>(ROWS ? a.llr_ch : a.ch_t) + fo;
    else ch = static_cast<const T *>(ROWS ? a.ch_a : a.ch_t) + fo;
    const T *la_in = static_cast<const T *>(ROWS ? a.la_rm : a.la_cm) + fo;
    T *la_out = static_cast<T *>(ROWS ? a.la_cm : a.la_rm) + fo;
    const uint32_t pos = LN::vn(line, hl, n);
    double lam = 0.0;
    if (live && hl < n) {
        T c;
        if (TOPO == kGldpc && first) c = static_cast<const T *>(a.llr_ch)[fo + pos];
        else c = ch[line * n + hl];
        lam = first ? (double)c : (double)c + (double)la_in[line * n + hl];
        if (first) {
            static_cast<T *>(a.ch_t)[fo + LN::cross(line, hl, n)] = c;
            if (TOPO == kGldpc) static_cast<T *>(a.ch_a)[fo + line * n + hl] = c;
        }
    }
    double lapp;
    const WordStats st = decode_pair<STOP>(a.code, a.L, a.qcap, a.pstop, lam, !live, S, lapp, lane,
                                           a.prof != nullptr);
    if (live && a.prof && hl == 0) prof_add(a.prof, st);
    const bool neg = live && hl < n && lapp < 0.0;
    const uint64_t hm = __ballot(neg);
    if (live && hl < n) {
        la_out[LN::cross(line, hl, n)] = (T)(a.alpha * (lapp - lam));
        if (a.llr_app) static_cast<T *>(a.llr_app)[fo + pos] = (T)lapp;
    }
    if (live && hl == 0) {
        a.masks[((size_t)f * n + line) * 2 + 0] = upper ? (hm >> 32) : (hm & 0xffffffffull);
        a.masks[((size_t)f * n + line) * 2 + 1] = 0ull;
        atomicAdd(reinterpret_cast<unsigned long long *>(&a.sumq[f]), (unsigned long long)st.Q);
        atomicMax(&a.halfmax[f], st.Q);
    }
}

// One wave per frame after half-iteration h: every word of the last pass and every
// word of the other family must have a zero syndrome.  A frame that finishes gets its
// hard decision from the last pass's line masks: element [j][c] (variable node j*n + c)
// is bit c of row j or bit j of column c of a product frame, bit j of word c of the
// first block row or of word (c - j) mod n of the second of a QC-GLDPC frame.
__global__ __launch_bounds__(kBlock) void k_product_check(ProductArgs a, int h, int last) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const size_t f = (size_t)blockIdx.x * kWavesPerBlock + wave;
    if (f >= a.nframes) return;
    if (a.done[f]) return;
    const int n = a.code.n;
    // the frame's line masks and the H columns are staged in LDS with coalesced loads,
    // so that the syndrome loops below read them without a memory access per bit
    __shared__ uint64_t mk_s[kWavesPerBlock][2 * SOGRAND_NMAX];
    __shared__ uint32_t hc_s[kWavesPerBlock][SOGRAND_NMAX];
    const uint64_t *mk_g = a.masks + f * n * 2;
    for (int t = lane; t < 2 * n; t += kWave) mk_s[wave][t] = mk_g[t];
    for (int t = lane; t < n; t += kWave) hc_s[wave][t] = a.code.hcol[t];
    wave_sync();
    const uint64_t *mk = mk_s[wave];
    const uint32_t *hcol = hc_s[wave];
    bool bad = false;
    if (a.topo == kProduct) {
        // Bit-sliced over the parity bits p: with Hp the positions whose H column has bit p,
        // line x's syndrome bit p is the parity of (line x AND Hp), and bit p of the cross
        // lines' syndromes, as a vector over them, is the XOR of the lines in Hp.  Lane t
        // holds lines t and t + 64 and the H columns of positions t and t + 64.
        const bool v0 = lane < n, v1 = lane + kWave < n;
        const uint64_t a0 = v0 ? mk[lane * 2] : 0ull, a1 = v0 ? mk[lane * 2 + 1] : 0ull;
        const uint64_t b0 = v1 ? mk[(lane + kWave) * 2] : 0ull, b1 = v1 ? mk[(lane + kWave) * 2 + 1] : 0ull;
        const uint32_t h0 = v0 ? hcol[lane] : 0u, h1 = v1 ? hcol[lane + kWave] : 0u;
        uint32_t used = h0 | h1;
        used |= xor_lane<1>(used);
        used |= xor_lane<2>(used);
        used |= xor_lane<4>(used);
        used |= xor_lane<8>(used);
        used |= xor_lane<16>(used);
        used |= xor_lane<32>(used);
        used = __builtin_amdgcn_readfirstlane(used);   // the parity bits present
        for (int p = 0; p < 32; p++) {
            if (!((used >> p) & 1u)) continue;
            const bool i0 = (h0 >> p) & 1u, i1 = (h1 >> p) & 1u;
            const uint64_t P0 = __ballot(i0), P1 = __ballot(i1);
            bad |= ((__popcll(a0 & P0) + __popcll(a1 & P1)) & 1) != 0;
            bad |= ((__popcll(b0 & P0) + __popcll(b1 & P1)) & 1) != 0;
            const uint64_t c0 = (i0 ? a0 : 0ull) ^ (i1 ? b0 : 0ull), c1 = (i0 ? a1 : 0ull) ^ (i1 ? b1 : 0ull);
            bad |= (wave_xor((uint32_t)c0) | wave_xor((uint32_t)(c0 >> 32)) | wave_xor((uint32_t)c1) |
                    wave_xor((uint32_t)(c1 >> 32))) != 0u;
        }
    }
    for (int b = 0; b < 2 && a.topo != kProduct; b++) {
        const int x = lane + kWave * b;
        if (x >= n) continue;
        // x as a line of the last pass: XOR of the columns of its set bits
        const uint64_t m0 = mk[x * 2], m1 = mk[x * 2 + 1];
        uint32_t s = 0;
        for (int i = 0; i < n; i++) {
            const uint64_t bit = i < 64 ? (m0 >> i) & 1ull : (m1 >> (i - 64)) & 1ull;
            if (bit) s ^= hcol[i];
        }
        // x as a word of the other family: its bit l is bit `bit` of the last pass's
        // word `src` (product: bit x of word l; QC-GLDPC: bit l of word (x + l) mod n
        // after a first-family pass, (x - l) mod n after a second-family pass)
        uint32_t t = 0;
        for (int l = 0; l < n; l++) {
            const int src = a.topo == kProduct ? l : ((h & 1) ? (x + l) % n : (x - l + n) % n);
            const int bit = a.topo == kProduct ? x : l;
            const uint64_t w = bit < 64 ? mk[src * 2] : mk[src * 2 + 1];
            if ((w >> (bit & 63)) & 1ull) t ^= hcol[l];
        }
        bad |= (s != 0u) || (t != 0u);
    }
    const bool valid = __ballot(bad) == 0ull;
    const bool finish = (valid && a.early_stop) || last;
    if (finish) {
        const bool rows = (h & 1) != 0;
        uint8_t *hd = a.hard + f * n * n;
        for (int j = 0; j < n; j++) {
            for (int c = lane; c < n; c += kWave) {
                int line, bit;
                if (a.topo == kProduct) {
                    line = rows ? j : c;
                    bit = rows ? c : j;
                } else {
                    bit = j;
                    line = rows ? c : (c >= j ? c - j : c - j + n);
                }
                hd[j * n + c] = (uint8_t)((mk[line * 2 + (bit >> 6)] >> (bit & 63)) & 1ull);
            }
        }
    }
    if (lane == 0) {
        a.summax[f] += a.halfmax[f];
        a.halfmax[f] = 0u;
        if (finish) {
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

// Workgroups of kWavesPerBlock waves (measured best on MI355X against 1 and 2), in
// plain dispatch order.  An XCD-aware order (consecutive lines of a frame on one XCD)
// measured slower: frames of similar SNR then share an XCD and its load.
static size_t word_grid(size_t words) { return (words + kWavesPerBlock - 1) / kWavesPerBlock; }

template <typename T, bool STOP>
static void launch_component_s(const ComponentArgs &a, int ns, dim3 g, hipStream_t st) {
    constexpr int W = kWavesPerBlock;
    if (ns == 32) hipLaunchKernelGGL((k_component<T, 32, W, STOP>), g, dim3(kWave * W), 0, st, a);
    else if (ns == 64) hipLaunchKernelGGL((k_component<T, 64, W, STOP>), g, dim3(kWave * W), 0, st, a);
    else hipLaunchKernelGGL((k_component<T, 128, W, STOP>), g, dim3(kWave * W), 0, st, a);
}

// the list-BLER stop is a separate instantiation, so that words without it pay nothing
template <typename T>
static void launch_component(const ComponentArgs &a, int ns, dim3 g, hipStream_t st) {
    if (a.pstop > 0.0) launch_component_s<T, true>(a, ns, g, st);
    else launch_component_s<T, false>(a, ns, g, st);
}

template <typename T, bool ROWS, bool STOP, int TOPO>
static void launch_pass_t(const ProductArgs &a, int ns, dim3 g, hipStream_t st) {
    constexpr int W = kWavesPerBlock;
    if (ns == 32) hipLaunchKernelGGL((k_product_pass_pair<T, ROWS, W, STOP, TOPO>), g, dim3(kWave * W), 0, st, a);
    else if (ns == 64) hipLaunchKernelGGL((k_product_pass<T, 64, ROWS, W, STOP, TOPO>), g, dim3(kWave * W), 0, st, a);
    else hipLaunchKernelGGL((k_product_pass<T, 128, ROWS, W, STOP, TOPO>), g, dim3(kWave * W), 0, st, a);
}

template <typename T, bool ROWS>
static void launch_pass(const ProductArgs &a, int ns, dim3 g, hipStream_t st) {
    if (a.topo == kProduct) {
        if (a.pstop > 0.0) launch_pass_t<T, ROWS, true, kProduct>(a, ns, g, st);
        else launch_pass_t<T, ROWS, false, kProduct>(a, ns, g, st);
    } else {
        if (a.pstop > 0.0) launch_pass_t<T, ROWS, true, kGldpc>(a, ns, g, st);
        else launch_pass_t<T, ROWS, false, kGldpc>(a, ns, g, st);
    }
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
    a.pstop = params->list_bler_stop;
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
    const size_t blocks = word_grid(nwords);
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

}  // extern "C"

namespace sg {

// Byte layout of the plain path's work buffer for nframes frames of length n:
// ch_t | la_rm | la_cm | [ch_a] | masks | done | halfmax | sumq | summax | half_iters.
struct WorkLayout {
    size_t ct, lr, lc, ca, mk, dn, hm, sq, sm, hi, total;
};

static WorkLayout work_layout(int topo, size_t nframes, int n, size_t esz) {
    WorkLayout w;
    const size_t plane = (nframes * n * n * esz + 255) & ~(size_t)255;
    w.ct = 0;
    w.lr = plane;
    w.lc = 2 * plane;
    w.ca = 3 * plane;
    w.mk = (topo == kGldpc ? 4 : 3) * plane;
    w.dn = (w.mk + nframes * n * 2 * sizeof(uint64_t) + 255) & ~(size_t)255;
    w.hm = (w.dn + nframes * sizeof(uint32_t) + 255) & ~(size_t)255;
    w.sq = (w.hm + nframes * sizeof(uint32_t) + 255) & ~(size_t)255;
    w.sm = (w.sq + nframes * sizeof(uint64_t) + 255) & ~(size_t)255;
    w.hi = (w.sm + nframes * sizeof(uint64_t) + 255) & ~(size_t)255;
    w.total = w.hi + nframes * sizeof(uint16_t);
    return w;
}

// Argument checks shared by the product and QC-GLDPC entry points.
static int check_frames(const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes,
                        const void *llr_ch, const uint8_t *hard, const uint8_t *success) {
    SG_TRY(check_params(params));
    if (!code) return fail(SOGRAND_EINVAL, "code is NULL");
    if (nframes == 0) return SOGRAND_OK;
    if (!llr_ch || !hard || !success) return fail(SOGRAND_EINVAL, "llr_ch, hard and success are required");
    const int n = code->n;
    const size_t words = nframes * (size_t)n;
    if (nframes > ((size_t)1 << 34) / ((size_t)n * n) || words >= ((size_t)1 << 31))
        return fail(SOGRAND_EINVAL, "nframes too large");
    return SOGRAND_OK;
}

// The block turbo loop over either family layout (see Lines), in the work buffer ws
// laid out by work_layout; `prof` false launches without the measurement hooks.
static int run_frames(int topo, const DevCode &dc, const sogrand_params_t *params, size_t nframes,
                      const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success, uint16_t *half_iters,
                      uint64_t *sum_queries, uint64_t *sum_max_queries, char *ws, hipStream_t st, bool prof) {
    const int n = dc.n;
    const size_t words = nframes * (size_t)n;
    const int ns = sort_width(n);
    // words of up to 32 bits go two to a wave
    const size_t blocks = word_grid(ns == 32 ? (words + 1) / 2 : words);
    const size_t esz = params->precision == SOGRAND_F64 ? sizeof(double) : sizeof(float);
    const WorkLayout w = work_layout(topo, nframes, n, esz);
    ProductArgs a;
    a.code = dc;
    a.L = params->list_max;
    a.qcap = params->query_cap;
    a.pstop = params->list_bler_stop;
    a.alpha = params->alpha;
    a.nframes = nframes;
    a.llr_ch = llr_ch;
    a.ch_t = ws + w.ct;
    a.la_rm = ws + w.lr;
    a.la_cm = ws + w.lc;
    a.ch_a = topo == kGldpc ? ws + w.ca : nullptr;
    a.first = 0;
    a.topo = topo;
    a.llr_app = llr_app;
    a.hard = hard;
    a.masks = reinterpret_cast<uint64_t *>(ws + w.mk);
    a.done = reinterpret_cast<uint32_t *>(ws + w.dn);
    a.halfmax = reinterpret_cast<uint32_t *>(ws + w.hm);
    a.sumq = sum_queries ? sum_queries : reinterpret_cast<uint64_t *>(ws + w.sq);
    a.summax = sum_max_queries ? sum_max_queries : reinterpret_cast<uint64_t *>(ws + w.sm);
    a.success = success;
    a.half_iters = half_iters ? half_iters : reinterpret_cast<uint16_t *>(ws + w.hi);
    a.early_stop = params->early_stop ? 1 : 0;
    a.prof = prof ? prof_counters(PK_PASS) : nullptr;
    const bool f64 = params->precision == SOGRAND_F64;
    const size_t ib = (nframes + kBlock - 1) / kBlock;
    const unsigned ig = (unsigned)(ib < 65536 ? ib : 65536);
    int tok = prof ? prof_start(PK_INIT, st) : -1;
    hipLaunchKernelGGL(k_product_init, dim3(ig), dim3(kBlock), 0, st, a);
    prof_stop(tok, st);
    const unsigned cg = (unsigned)((nframes + kWavesPerBlock - 1) / kWavesPerBlock);
    for (int h = 1; h <= 2 * params->max_iter; h++) {
        const bool rows = (h & 1) != 0;
        a.first = h == 1 ? 1 : 0;
        tok = prof ? prof_start(PK_PASS, st) : -1;
        if (f64) {
            if (rows) launch_pass<double, true>(a, ns, dim3((unsigned)blocks), st);
            else launch_pass<double, false>(a, ns, dim3((unsigned)blocks), st);
        } else {
            if (rows) launch_pass<float, true>(a, ns, dim3((unsigned)blocks), st);
            else launch_pass<float, false>(a, ns, dim3((unsigned)blocks), st);
        }
        prof_stop(tok, st);
        tok = prof ? prof_start(PK_CHECK, st) : -1;
        hipLaunchKernelGGL(k_product_check, dim3(cg), dim3(kBlock), 0, st, a, h, h == 2 * params->max_iter ? 1 : 0);
        prof_stop(tok, st);
    }
    if (hipGetLastError() != hipSuccess) return fail(SOGRAND_EDEVICE, "product kernel launch failed");
    return SOGRAND_OK;
}

static int decode_frames(int topo, const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes,
                         const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                         uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries, void *stream) {
    SG_TRY(check_frames(code, params, nframes, llr_ch, hard, success));
    if (nframes == 0) return SOGRAND_OK;
    DevCode dc;
    SG_TRY(prepare_code(const_cast<sogrand_code_t *>(code), params->query_cap, &dc));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t esz = params->precision == SOGRAND_F64 ? sizeof(double) : sizeof(float);
    const WorkLayout w = work_layout(topo, nframes, code->n, esz);
    char *ws = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&ws), w.total, st) != hipSuccess)
        return fail(SOGRAND_ENOMEM, "work buffer allocation of %zu bytes failed", w.total);
    const int rc = run_frames(topo, dc, params, nframes, llr_ch, hard, llr_app, success, half_iters, sum_queries,
                              sum_max_queries, ws, st, true);
    (void)hipFreeAsync(ws, st);
    return rc;
}

// ----------------------------------------------------------------------------
// the product path without allocation: the work buffer is a static device array
// ----------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)SOGRAND_NOALLOC_WORK_MAX;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices];   // the array's device address on each device, once looked up

// The address of this device's copy of `scratch`.  In host code the array's name is
// only a stand-in for the symbol, so the address is looked up once per device and
// used from then on.
static int scratch_address(void **out) {
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SOGRAND_EDEVICE, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SOGRAND_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SOGRAND_OK;
}

}  // namespace sg

// A decode's launches recorded once (see sogrand_plan_create): the graph and the work
// buffer that its kernels address.
struct sogrand_plan {
    int device = 0;
    char *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace sg {

static void plan_free(sogrand_plan *p) {
    if (!p) return;
    if (p->exec) {
        // replays still running use the work buffer: wait for the plan's device first
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (have && cur != p->device) (void)hipSetDevice(p->device);
        (void)hipDeviceSynchronize();
        if (have && cur != p->device) (void)hipSetDevice(cur);
        (void)hipGraphExecDestroy(p->exec);
    }
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
}

// Records run_frames on a capture stream of its own: the initialisation and, per
// half-iteration, the pass and the validity check, all kernels (no memory set or copy
// nodes), addressing a work buffer that the plan owns.
static int plan_create(int topo, const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes,
                       const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success, uint16_t *half_iters,
                       uint64_t *sum_queries, uint64_t *sum_max_queries, sogrand_plan **out) {
    if (!out) return fail(SOGRAND_EINVAL, "out is NULL");
    *out = nullptr;
    SG_TRY(check_frames(code, params, nframes, llr_ch, hard, success));
    if (nframes == 0) return fail(SOGRAND_EINVAL, "a plan needs at least one frame");
    DevCode dc;
    SG_TRY(prepare_code(const_cast<sogrand_code_t *>(code), params->query_cap, &dc));
    sogrand_plan *p = new (std::nothrow) sogrand_plan;
    if (!p) return fail(SOGRAND_ENOMEM, "plan");
    if (hipGetDevice(&p->device) != hipSuccess) {
        plan_free(p);
        return fail(SOGRAND_EDEVICE, "hipGetDevice failed");
    }
    const size_t esz = params->precision == SOGRAND_F64 ? sizeof(double) : sizeof(float);
    const WorkLayout w = work_layout(topo, nframes, code->n, esz);
    if (hipMalloc(reinterpret_cast<void **>(&p->ws), w.total) != hipSuccess) {
        plan_free(p);
        return fail(SOGRAND_ENOMEM, "work buffer allocation of %zu bytes failed", w.total);
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        plan_free(p);
        return fail(SOGRAND_EDEVICE, "capture stream creation failed");
    }
    int rc = SOGRAND_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = fail(SOGRAND_EDEVICE, "hipStreamBeginCapture failed");
    } else {
        rc = run_frames(topo, dc, params, nframes, llr_ch, hard, llr_app, success, half_iters, sum_queries,
                        sum_max_queries, p->ws, cs, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        p->graph = g;
        if (rc == SOGRAND_OK && (e != hipSuccess || !g)) rc = fail(SOGRAND_EDEVICE, "graph capture failed");
    }
    (void)hipStreamDestroy(cs);
    if (rc == SOGRAND_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(SOGRAND_EDEVICE, "hipGraphInstantiate failed");
    if (rc != SOGRAND_OK) {
        plan_free(p);
        return rc;
    }
    *out = p;
    return SOGRAND_OK;
}

}  // namespace sg

extern "C" {

int sogrand_plan_create(const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes, int gldpc,
                        const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success, uint16_t *half_iters,
                        uint64_t *sum_queries, uint64_t *sum_max_queries, sogrand_plan_t **out) {
    return sg::plan_create(gldpc ? sg::kGldpc : sg::kProduct, code, params, nframes, llr_ch, hard, llr_app, success,
                           half_iters, sum_queries, sum_max_queries, out);
}

int sogrand_plan_launch(sogrand_plan_t *plan, void *stream) {
    using namespace sg;
    if (!plan) return fail(SOGRAND_EINVAL, "plan is NULL");
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(SOGRAND_EINVAL, "the plan was made on device %d, not %d", plan->device, dev);
    SG_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return SOGRAND_OK;
}

void sogrand_plan_destroy(sogrand_plan_t *plan) {
    sg::plan_free(plan);
}

int sogrand_decode_product(const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes,
                           const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                           uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                           void *stream) {
    return sg::decode_frames(sg::kProduct, code, params, nframes, llr_ch, hard, llr_app, success, half_iters,
                             sum_queries, sum_max_queries, stream);
}

int sogrand_decode_gldpc(const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes,
                         const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                         uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                         void *stream) {
    return sg::decode_frames(sg::kGldpc, code, params, nframes, llr_ch, hard, llr_app, success, half_iters,
                             sum_queries, sum_max_queries, stream);
}

int sogrand_decode_product_noalloc(const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes,
                                   const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                                   uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                                   void *stream) {
    using namespace sg;
    SG_TRY(check_frames(code, params, nframes, llr_ch, hard, success));
    if (nframes == 0) return SOGRAND_OK;
    const size_t esz = params->precision == SOGRAND_F64 ? sizeof(double) : sizeof(float);
    const WorkLayout w = work_layout(kProduct, nframes, code->n, esz);
    if (w.total > kScratchBytes)
        return fail(SOGRAND_EINVAL, "%zu frames need %zu bytes of work buffer, above the %zu of the static buffer",
                    nframes, w.total, kScratchBytes);
    DevCode dc;
    SG_TRY(prepare_code(const_cast<sogrand_code_t *>(code), params->query_cap, &dc, false));
    void *ws = nullptr;
    SG_TRY(scratch_address(&ws));
    return run_frames(kProduct, dc, params, nframes, llr_ch, hard, llr_app, success, half_iters, sum_queries,
                      sum_max_queries, static_cast<char *>(ws), static_cast<hipStream_t>(stream), false);
}

}  // extern "C"
