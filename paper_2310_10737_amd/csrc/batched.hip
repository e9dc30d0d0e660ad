// Batched block-turbo decoding of product or QC-GLDPC frames of mixed codes in
// one persistent launch.
//
// Each workgroup owns up to `slots` frames at a time (frame slots in LDS).  Its
// waves steal ranges of `chunk` lines of the current half-iteration of any of
// those frames through LDS atomics, decode them (one wave per line, as in the
// plain path), and report.  The wave that finishes the last line of a half
// tests the hard decision (every row and column a codeword, section "Iterative
// decoding"), then either opens the next half-iteration or writes the frame's
// results and refills the slot from one global frame counter.  All
// coordination is workgroup-local, so no cache maintenance across XCDs is
// needed; frames are independent, so the result of a frame does not depend on
// the schedule.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "pair.hpp"

namespace sg {

constexpr int kMaxCodes = 8;
constexpr int kMaxSlots = 8;
constexpr uint32_t kSpinLimit = 1u << 26;   // idle scans before a wave reports a stall

struct CodeTable {
    DevCode codes[kMaxCodes];
};

struct BatchArgs {
    const DevCode *codes;           // [ncodes], in device memory
    int ncodes;
    int topo;                       // kProduct or kGldpc: every frame of the batch
    int L;
    uint32_t qcap;
    double pstop;                   // list-BLER stop threshold, 0 = off
    double alpha;
    int max_iter;
    int early_stop;
    uint32_t nframes;
    const uint8_t *frame_code;      // [F]
    const uint64_t *frame_offset;   // [F] element offset of the frame's n x n block
    uint64_t llr_len;               // elements of llr_ch / hard
    const void *llr_ch;
    uint8_t *hard;
    void *llr_app;                  // optional, written every half-iteration (the last one stays)
    uint8_t *success;
    uint16_t *half_iters;
    uint64_t *sumq;
    uint64_t *summax;
    void *la;                       // [grid][slots][nmax * nmax]
    int nmax;
    int slots;
    int chunk;
    uint32_t *next_frame;           // global frame counter
    const uint32_t *order;          // [F] frame taken at each count (longest codes, then hardest frames, first)
    uint32_t *error;                // bit 0: a wave stopped waiting; bit 1: a frame descriptor was invalid
    uint32_t *status;               // caller's copy of the error bits, or NULL
    ProfCounters *prof;
};

struct SlotLds {
    uint64_t masks[SOGRAND_NMAX][2];   // hard decision of each line of the current half
    unsigned long long sumq, summax;
    // claim word: generation (bits 63..40), lines of the half n (39..32) and the next
    // unclaimed line (31..0).  A claim and the n it is judged against come from one
    // atomic; the generation changes whenever the slot opens a new half-iteration.
    unsigned long long ctl;
    int frame;       // frame index; -1: no frame left (retired)
    int code;
    int n;
    int h;           // current half-iteration, 1 .. 2 max_iter
    int done;        // lines of this half finished
    unsigned int halfmax;
};

__device__ __forceinline__ unsigned long long ctl_word(unsigned long long gen, int n) {
    return (gen << 40) | ((unsigned long long)(n & 0xff) << 32);
}

__device__ __forceinline__ int lds_load(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ unsigned long long lds_load64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Opens the slot's next half-iteration (or retires it) after its fields are set.
__device__ __forceinline__ void slot_publish(SlotLds &sl) {
    const unsigned long long gen = (sl.ctl >> 40) + 1;
    const int n = sl.frame >= 0 ? sl.n : 0;
    __hip_atomic_store(&sl.ctl, ctl_word(gen, n), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Takes the next frame for slot `sl` (single lane).  Invalid descriptors are
// reported and the frame is skipped with success 0 and zero half-iterations.
__device__ void slot_refill(const BatchArgs &a, SlotLds &sl) {
    for (;;) {
        const uint32_t k = atomicAdd(a.next_frame, 1u);
        if (k >= a.nframes) {
            sl.frame = -1;
            return;
        }
        const uint32_t f = a.order ? a.order[k] : k;
        const int code = a.frame_code[f];
        const int n = code < a.ncodes ? a.codes[code].n : 0;
        const uint64_t off = a.frame_offset[f];
        if (code >= a.ncodes || off > a.llr_len || a.llr_len - off < (uint64_t)n * n) {
            atomicOr(a.error, 2u);
            a.success[f] = 0;
            if (a.half_iters) a.half_iters[f] = 0;
            if (a.sumq) a.sumq[f] = 0;
            if (a.summax) a.summax[f] = 0;
            continue;
        }
        sl.frame = (int)f;
        sl.code = code;
        sl.n = n;
        sl.h = 1;
        sl.done = 0;
        sl.halfmax = 0;
        sl.sumq = 0;
        sl.summax = 0;
        return;
    }
}

// Validity of the frame's hard decision after half-iteration h: every line of
// the last pass and every line of the other family has a zero syndrome.  The
// masks hold the last pass's lines.  Bit l of the other family's word x is, for a
// product code, bit x of line l; for a QC-GLDPC code, bit l of line (x + l) mod n
// after a first-family pass and of line (x - l) mod n after a second-family pass
// (both families take bit l from block l).  The H columns are staged in the wave's
// own LDS scratch (its list-membership words, which the next decode clears), so the
// loops below read LDS, without a dependent global load per bit.
template <int TOPO>
__device__ __forceinline__ bool slot_valid(const SlotLds &sl, const DevCode &c, WaveLds &S, int lane, int h) {
    const int n = sl.n;
    if constexpr (TOPO == kProduct) {
        // Bit-sliced over the parity bits p: with Hp the positions whose H column has bit p,
        // line x's syndrome bit p is the parity of (line x AND Hp), and bit p of the cross
        // lines' syndromes, as a vector over them, is the XOR of the lines in Hp.  Lane t
        // holds lines t and t + 64 and the H columns of positions t and t + 64.
        const bool v0 = lane < n, v1 = lane + kWave < n;
        const uint64_t a0 = v0 ? sl.masks[lane][0] : 0ull, a1 = v0 ? sl.masks[lane][1] : 0ull;
        const uint64_t b0 = v1 ? sl.masks[lane + kWave][0] : 0ull, b1 = v1 ? sl.masks[lane + kWave][1] : 0ull;
        const uint32_t h0 = v0 ? gptr(c.hcol)[lane] : 0u, h1 = v1 ? gptr(c.hcol)[lane + kWave] : 0u;
        uint32_t used = h0 | h1;
        used |= xor_lane<1>(used);
        used |= xor_lane<2>(used);
        used |= xor_lane<4>(used);
        used |= xor_lane<8>(used);
        used |= xor_lane<16>(used);
        used |= xor_lane<32>(used);
        used = __builtin_amdgcn_readfirstlane(used);   // the parity bits present
        bool bad = false;
#pragma unroll 1
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
        return __ballot(bad) == 0ull;
    }
    uint32_t *hc = S.zmask;
    for (int t = lane; t < n; t += kWave) hc[t] = gptr(c.hcol)[t];
    wave_sync();
    bool bad = false;
    for (int b = 0; b < 2; b++) {
        const int x = lane + kWave * b;
        if (x >= n) continue;
        const uint64_t m0 = sl.masks[x][0], m1 = sl.masks[x][1];
        const int half = x >> 6, xb = x & 63;
        uint32_t s = 0, t = 0;
        if constexpr (TOPO == kProduct) {
#pragma unroll 1
            for (int l = 0; l < n; l++) {
                const uint32_t col = hc[l];
                const uint64_t own = l < 64 ? m0 >> l : m1 >> (l - 64);
                s ^= col & (0u - (uint32_t)(own & 1ull));
                t ^= col & (0u - (uint32_t)((sl.masks[l][half] >> xb) & 1ull));
            }
        } else {
            const bool after_first = (h & 1) != 0;
#pragma unroll 1
            for (int l = 0; l < n; l++) {
                const uint32_t col = hc[l];
                const uint64_t own = l < 64 ? m0 >> l : m1 >> (l - 64);
                s ^= col & (0u - (uint32_t)(own & 1ull));
                int src = after_first ? x + l : x - l;
                if (src >= n) src -= n;
                if (src < 0) src += n;
                const uint64_t w = l < 64 ? sl.masks[src][0] : sl.masks[src][1];
                t ^= col & (0u - (uint32_t)((w >> (l & 63)) & 1ull));
            }
        }
        bad |= (s != 0u) || (t != 0u);
    }
    return __ballot(bad) == 0ull;
}

// Decodes line `line` of the slot's frame in half-iteration h: a word of the
// first family (product rows, the first block row of a QC-GLDPC code) for odd h,
// of the second otherwise.  Frame positions are variable nodes: bit i of a
// product row is line*n + i, of a column i*n + line; bit i of a QC-GLDPC word is
// i*n + line in the first block row and i*n + (line + i) mod n in the second.
template <typename T, int NS, bool STOP, int TOPO, bool LDSLOG>
__device__ __forceinline__ WordStats batch_line(const BatchArgs &a, SlotLds &sl, const DevCode &c,
                                                const DevCode *cdev, int frame,
                                                int h, int line, T *la, WaveLds &S, int lane) {
    constexpr int NB = Lanes<NS>::NB;
    const int n = c.n;
    const bool rows = (h & 1) != 0;
    const uint64_t off = load_uniform(a.frame_offset + frame);
    const T *ch = static_cast<const T *>(a.llr_ch) + off;
    double lam[NB];
    int pos[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        if constexpr (TOPO == kProduct) {
            pos[b] = rows ? line * n + i : i * n + line;
        } else {
            int col = rows ? line : line + i;
            if (col >= n) col -= n;
            pos[b] = i * n + col;
        }
        // the a-priori LLRs are zero in the first half-iteration
        lam[b] = i < n ? (double)ch[pos[b]] + (h > 1 ? (double)la[pos[b]] : 0.0) : 0.0;
    }
    double lapp[NB];
    const WordStats st = decode_word<NS, true, STOP, LDSLOG>(c, cdev, a.L, a.qcap, a.pstop, lam, S, lapp, lane,
                                                     a.prof != nullptr);
    uint64_t hm[2] = {0ull, 0ull};
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        const bool v = i < n;
        const bool neg = v && lapp[b] < 0.0;
        hm[b] = __ballot(neg);
        if (!v) continue;
        la[pos[b]] = (T)(a.alpha * (lapp[b] - lam[b]));
        if (a.llr_app) static_cast<T *>(a.llr_app)[off + pos[b]] = (T)lapp[b];
    }
    if (lane == 0) {
        sl.masks[line][0] = hm[0];
        sl.masks[line][1] = hm[1];
    }
    return st;
}

// Decodes lines `line` (lanes 0-31) and `line + 1` (lanes 32-63) of the slot's frame
// in half-iteration h, two words of up to 32 bits per wave (decode_pair), at the
// same frame positions as batch_line.  A half whose line is not below `last` takes
// part without testing patterns.
template <typename T, bool STOP, int TOPO>
__device__ __forceinline__ WordStats batch_pair(const BatchArgs &a, SlotLds &sl, const DevCode &c, int frame, int h,
                                                int line, int last, T *la, PairLds *P, int lane) {
    const int n = c.n;
    const bool rows = (h & 1) != 0;
    const int hl = lane & 31;
    const bool upper = lane >= 32;
    const int ln = line + (upper ? 1 : 0);
    const bool live = ln < last;
    const uint64_t off = load_uniform(a.frame_offset + frame);
    const T *ch = static_cast<const T *>(a.llr_ch) + off;
    int pos;
    if constexpr (TOPO == kProduct) {
        pos = rows ? ln * n + hl : hl * n + ln;
    } else {
        int col = rows ? ln : ln + hl;
        if (col >= n) col -= n;
        pos = hl * n + col;
    }
    const bool v = live && hl < n;
    const double lam = v ? (double)ch[pos] + (h > 1 ? (double)la[pos] : 0.0) : 0.0;
    double lapp;
    const WordStats st = decode_pair<STOP, true>(c, a.L, a.qcap, a.pstop, lam, !live, P[upper ? 1 : 0], lapp, lane,
                                                 a.prof != nullptr);
    const bool neg = v && lapp < 0.0;
    const uint64_t hm = __ballot(neg);
    if (v) {
        la[pos] = (T)(a.alpha * (lapp - lam));
        if (a.llr_app) static_cast<T *>(a.llr_app)[off + pos] = (T)lapp;
    }
    if (live && hl == 0) {
        sl.masks[ln][0] = upper ? (hm >> 32) : (hm & 0xffffffffull);
        sl.masks[ln][1] = 0ull;
    }
    return st;
}

// The frame's hard decision, written once when it retires: bit `bit` of line `line`'s
// mask after half-iteration h is the decision on that word's bit, and element [j][c]
// (variable node j*n + c) is bit c of row j or bit j of column c of a product frame, bit j
// of word c of the first block row or of word (c - j) mod n of the second of a QC-GLDPC
// frame.  Consecutive lanes write consecutive bytes of a row of the frame.
template <int TOPO>
__device__ __forceinline__ void write_hard(uint8_t *hard, const SlotLds &sl, int n, int h, int lane) {
    const bool rows = (h & 1) != 0;
    for (int j = 0; j < n; j++) {
        for (int c = lane; c < n; c += kWave) {
            int line, bit;
            if constexpr (TOPO == kProduct) {
                line = rows ? j : c;
                bit = rows ? c : j;
            } else {
                bit = j;
                line = rows ? c : (c >= j ? c - j : c - j + n);
            }
            const uint64_t w = sl.masks[line][bit >> 6];
            hard[j * n + c] = (uint8_t)((w >> (bit & 63)) & 1ull);
        }
    }
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

// Waves per SIMD that the register allocation of each instantiation aims at: eight for
// product frames of up to 64 bits without the list-BLER stop (64 registers, no spills),
// six otherwise (the 128-bit instantiations spill a few registers there and still beat
// four waves with none; the stop and QC-GLDPC forms of the 64-bit one would spill more
// at eight).
template <int NSMAX, bool STOP, int TOPO>
constexpr int batched_waves() {
    return NSMAX == 64 && !STOP && TOPO == kProduct ? 8 : 6;
}

// NSMAX: 32 when every code of the batch has n <= 32 (two words per wave), 64 when
// n <= 64, else 128; the narrower instantiations compile without the wider paths.
template <typename T, int WPB, int NSMAX, bool STOP, int TOPO>
__global__ __launch_bounds__(kWave * WPB) __attribute__((amdgpu_waves_per_eu(batched_waves<NSMAX, STOP, TOPO>())))
void k_batched(BatchArgs a) {
    __shared__ WaveLds wl[WPB];
    extern __shared__ SlotLds slot_dyn[];
    SlotLds *sls = slot_dyn;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    WaveLds &S = wl[wave];
    const int nslots = a.slots;
    if (threadIdx.x == 0)
        for (int s = 0; s < nslots; s++) {
            sls[s].ctl = 0ull;
            slot_refill(a, sls[s]);
            slot_publish(sls[s]);
        }
    // the 128-bit instantiations (6 waves per SIMD) read the logarithm's table from LDS; at the
    // 64-bit one's 8 waves the table reads added to the query loop's LDS traffic cost more
    if constexpr (NSMAX == 128) fill_log_table();
    __syncthreads();
    T *la_base = static_cast<T *>(a.la) + (size_t)blockIdx.x * nslots * a.nmax * a.nmax;
    uint32_t idle = 0;
#ifdef SG_PHASE_CLOCKS
    ProfAcc acc;   // the clocked build adds its counters up once, when the wave ends
#endif
#ifdef SG_PHASE_CLOCKS
    uint64_t t_free = __builtin_amdgcn_s_memtime();   // end of this wave's last line of work
#endif
    int start = wave % nslots;
    for (;;) {
        // steal a range of lines from any slot with unclaimed lines
        int sel = -1, first = 0;
        bool live = false;
        for (int k = 0; k < nslots; k++) {
            const int s = (start + k) % nslots;
            SlotLds &sl = sls[s];
            if (lds_load(&sl.frame) < 0) continue;
            live = true;
            const unsigned long long c0 = lds_load64(&sl.ctl);
            if ((uint32_t)c0 >= (uint32_t)((c0 >> 32) & 0xff)) continue;   // nothing left to claim
            unsigned long long got = 0;
            if (lane == 0)
                got = __hip_atomic_fetch_add(&sl.ctl, (unsigned long long)a.chunk, __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)got);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
            if (lo < (hi & 0xffu)) {
                sel = s;
                first = (int)lo;
                break;
            }
        }
        if (sel < 0) {
            if (!live) break;
            if (++idle > kSpinLimit) {
                if (lane == 0) atomicOr(a.error, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        idle = 0;
        start = sel;
        SlotLds &sl = sls[sel];
        // a valid claim sees the fields written before its generation was published
        const int frame = __builtin_amdgcn_readfirstlane(lds_load(&sl.frame));
        const int code = __builtin_amdgcn_readfirstlane(sl.code);
        const int h = __builtin_amdgcn_readfirstlane(sl.h);
        const DevCode c = load_uniform(a.codes + code);
        const int n = c.n;
        const int last = first + a.chunk < n ? first + a.chunk : n;
        T *la = la_base + (size_t)sel * a.nmax * a.nmax;
        unsigned long long qsum = 0;
        uint32_t qmax = 0;
        if constexpr (NSMAX == 32) {
            static_assert(2 * sizeof(PairLds) <= sizeof(WaveLds), "two pair scratches per wave");
            PairLds *P = reinterpret_cast<PairLds *>(&S);
            for (int line = first; line < last; line += 2) {
                const WordStats st = batch_pair<T, STOP, TOPO>(a, sl, c, frame, h, line, last, la, P, lane);
                const bool live = line + (lane >= 32 ? 1 : 0) < last;
                if (live && a.prof && (lane & 31) == 0) prof_add(a.prof, st);
                if (live) {
                    qsum += st.Q;
                    qmax = st.Q > qmax ? st.Q : qmax;
                }
            }
            // the two halves' sums, for lane 0 to report
            qsum = readlane_u64(qsum, 0) + readlane_u64(qsum, 32);
            const uint32_t m0 = (uint32_t)__builtin_amdgcn_readlane((int)qmax, 0);
            const uint32_t m1 = (uint32_t)__builtin_amdgcn_readlane((int)qmax, 32);
            qmax = m0 > m1 ? m0 : m1;
        } else {
            for (int line = first; line < last; line++) {
                WordStats st;
                SG_CLOCK(l0);
                if (NSMAX == 64 || n <= 64) st = batch_line<T, 64, STOP, TOPO, NSMAX == 128>(a, sl, c, a.codes + code, frame, h, line, la, S, lane);
                else st = batch_line<T, 128, STOP, TOPO, NSMAX == 128>(a, sl, c, a.codes + code, frame, h, line, la, S, lane);
#ifdef SG_PHASE_CLOCKS
                SG_CLOCK(l1);
                uint32_t inner = 0;
                for (int q = 0; q < 5; q++) inner += st.phase[q];
                st.phase[5] = (uint32_t)(l1 - l0) - inner;
                // the time since this wave's previous line, less the line itself: finding work
                st.phase[6] = (uint32_t)(l0 - t_free);
                t_free = l1;
#endif
#ifdef SG_PHASE_CLOCKS
                if (a.prof) acc.add(st);
#else
                if (a.prof && lane == 0) prof_add(a.prof, st);
#endif
                qsum += st.Q;
                qmax = st.Q > qmax ? st.Q : qmax;
            }
        }
        // the lines' global writes complete before they are counted as done
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        int d = 0;
        if (lane == 0) {
            atomicAdd(&sl.sumq, qsum);
            atomicMax(&sl.halfmax, qmax);
            d = atomicAdd(&sl.done, last - first) + (last - first);
        }
        d = __builtin_amdgcn_readfirstlane(d);
        if (d != n) continue;

        // this wave finished the half-iteration
        SG_CLOCK(v0);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const bool valid = slot_valid<TOPO>(sl, c, S, lane, h);
        const bool retire = (valid && a.early_stop) || h == 2 * a.max_iter;
        if (retire) write_hard<TOPO>(a.hard + load_uniform(a.frame_offset + frame), sl, n, h, lane);
        if (lane == 0) {
            sl.summax += sl.halfmax;
            sl.halfmax = 0;
            if (retire) {
                a.success[frame] = valid;
                if (a.half_iters) a.half_iters[frame] = (uint16_t)h;
                if (a.sumq) a.sumq[frame] = sl.sumq;
                if (a.summax) a.summax[frame] = sl.summax;
                slot_refill(a, sl);
            } else {
                sl.h = h + 1;
                sl.done = 0;
            }
            slot_publish(sl);
        }
#ifdef SG_PHASE_CLOCKS
        // the hand-over is not time spent finding work
        SG_CLOCK(v1);
        acc.phase[7] += v1 - v0;
        t_free += v1 - v0;
#endif
    }
#ifdef SG_PHASE_CLOCKS
    if (a.prof && lane == 0) acc.flush(a.prof);
#endif
}

// Zeroes the frame counter and error bits and stores the code table where the
// persistent kernel reads it.
__global__ void k_batched_init(uint32_t *counters, CodeTable table, DevCode *dst, int ncodes) {
    if (threadIdx.x < 2) counters[threadIdx.x] = 0u;
    if (threadIdx.x < (unsigned)ncodes) dst[threadIdx.x] = table.codes[threadIdx.x];
}

// The order in which the persistent kernel takes frames: those of the longest codes
// first, so that the end of the launch, when waves run out of frames, is left to the
// shortest code; and the frames of that last code hardest first, judged by their mean
// channel reliability |L| (small means many unreliable bits, and so more queries and
// half-iterations), so that the launch ends on short, easy frames.  The frames of the
// other codes keep their input order: taking the hardest of them together, early on,
// gave slower launches, since the waves of a workgroup then more often wait on the
// long words of all of its frames at once.  Results do not depend on the order.
//
// k_frame_ease writes each frame's mean |L| over a sample of its first elements (one
// wave per frame; frames of other codes get 0, invalid descriptors -1); k_batched_order
// then sorts the frames by (rank of the code's length, ease level), the level being the
// frame's place between the smallest and largest ease among the last code's frames, cut
// into `levels` equal steps.  Descriptors that name no code or a block outside llr_ch,
// and frames whose sample holds a NaN, go last.
constexpr int kEaseSample = 1024;
constexpr int kOrderThreads = 512;
constexpr int kOrderBins = 24;   // one per code, plus the last code's extra levels and the invalid frames

struct OrderKeys {
    uint8_t rank[kMaxCodes];   // rank of each code index by length, longest first
    int n[kMaxCodes];          // length of each code index
    int ncodes;
    int last;                  // index of the code of rank ncodes - 1, whose frames are ordered by ease
    int levels;                // ease levels of the last code: ncodes + levels <= kOrderBins
};

template <typename T>
__global__ __launch_bounds__(256) void k_frame_ease(const uint8_t *frame_code, const uint64_t *frame_offset,
                                                    uint32_t nframes, uint64_t llr_len, const T *llr,
                                                    OrderKeys ok, float *ease) {
    const uint32_t f = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (f >= nframes) return;
    const uint32_t c = frame_code[f];
    const uint64_t off = frame_offset[f];
    float s = 0.f;
    uint32_t m = 0;
    bool valid = false;
    if (c < (uint32_t)ok.ncodes) {
        const uint64_t len = (uint64_t)ok.n[c] * ok.n[c];
        valid = off <= llr_len && llr_len - off >= len;
        if (valid && c == (uint32_t)ok.last) {
            m = len < (uint64_t)kEaseSample ? (uint32_t)len : (uint32_t)kEaseSample;
            for (uint32_t i0 = 0; i0 < m; i0 += 4 * kWave) {   // four loads in flight
                float v[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t i = i0 + u * kWave + lane;
                    v[u] = i < m ? fabsf((float)llr[off + i]) : 0.f;
                }
                s += (v[0] + v[1]) + (v[2] + v[3]);
            }
        }
    }
    for (int d = kWave / 2; d > 0; d >>= 1) s += __shfl_xor(s, d);
    if (lane == 0) ease[f] = !valid ? -1.f : m ? s / (float)m : 0.f;
}

__global__ __launch_bounds__(kOrderThreads) void k_batched_order(const uint8_t *frame_code, const float *ease,
                                                                 uint32_t nframes, OrderKeys ok, uint32_t *order) {
    constexpr int kWaves = kOrderThreads / kWave;
    constexpr int kBatch = 16;   // frames whose loads a thread has in flight together
    __shared__ uint32_t cnt[kOrderBins][kOrderThreads];   // frames per bin and thread, then positions
    __shared__ uint32_t wsum[kOrderBins][kWaves];
    __shared__ uint32_t base[kOrderBins];
    __shared__ float wlo[kWaves], whi[kWaves];
    __shared__ uint32_t rank_s[kMaxCodes];
    const uint32_t t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    const int nc = ok.ncodes, levels = ok.levels, nbins = nc + levels;
    const uint32_t last = (uint32_t)ok.last;
    // each thread takes frames t, t + kOrderThreads, ... in every pass below, and issues
    // the loads of kBatch of them before it uses them
    auto load = [&](uint32_t f0, uint32_t (&c)[kBatch], float (&e)[kBatch]) {
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
            const uint32_t f = f0 + u * kOrderThreads + t;
            c[u] = f < nframes ? frame_code[f] : 0xffu;
            e[u] = f < nframes ? ease[f] : -1.f;
        }
    };
    // the range of ease over the last code's frames
    float lo = INFINITY, hi = -INFINITY;
    for (uint32_t f0 = 0; f0 < nframes; f0 += kBatch * kOrderThreads) {
        uint32_t c[kBatch];
        float e[kBatch];
        load(f0, c, e);
#pragma unroll
        for (int u = 0; u < kBatch; u++)
            if (c[u] == last && e[u] >= 0.f) lo = fminf(lo, e[u]), hi = fmaxf(hi, e[u]);
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, d));
        hi = fmaxf(hi, __shfl_xor(hi, d));
    }
    if (lane == 0) wlo[wave] = lo, whi[wave] = hi;
    for (int b = 0; b < nbins; b++) cnt[b][t] = 0u;
    if (t < (uint32_t)nc) rank_s[t] = ok.rank[t];
    __syncthreads();
    for (int w = 0; w < kWaves; w++) lo = fminf(lo, wlo[w]), hi = fmaxf(hi, whi[w]);
    const float step = hi > lo ? (float)levels / (hi - lo) : 0.f;
    auto bin = [&](uint32_t c, float e) -> uint32_t {
        if (c >= (uint32_t)nc || !(e >= 0.f)) return (uint32_t)(nbins - 1);
        if (c != last) return rank_s[c];
        const float r = (e - lo) * step;
        const int lv = r < (float)levels ? (int)fmaxf(r, 0.f) : levels - 1;   // NaN lands on the last level
        return (uint32_t)(nc - 1 + lv);
    };
    for (uint32_t f0 = 0; f0 < nframes; f0 += kBatch * kOrderThreads) {
        uint32_t c[kBatch];
        float e[kBatch];
        load(f0, c, e);
#pragma unroll
        for (int u = 0; u < kBatch; u++)
            if (f0 + u * kOrderThreads + t < nframes) cnt[bin(c[u], e[u])][t]++;
    }
    // exclusive prefix of each bin's counts over the threads: within each wave by
    // shuffles, then over the waves' totals, then over the bins
    for (int b = 0; b < nbins; b++) {
        const uint32_t v = cnt[b][t];
        uint32_t incl = v;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)incl, d);
            if (lane >= (uint32_t)d) incl += u;
        }
        cnt[b][t] = incl - v;
        if (lane == kWave - 1) wsum[b][wave] = incl;
    }
    __syncthreads();
    if (t < (uint32_t)nbins) {
        uint32_t acc = 0;
        for (int w = 0; w < kWaves; w++) {
            const uint32_t x = wsum[t][w];
            wsum[t][w] = acc;
            acc += x;
        }
        base[t] = acc;   // the bin's total, made a base below
    }
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < nbins; b++) {
            const uint32_t x = base[b];
            base[b] = acc;
            acc += x;
        }
    }
    __syncthreads();
    for (int b = 0; b < nbins; b++) cnt[b][t] += base[b] + wsum[b][wave];
    for (uint32_t f0 = 0; f0 < nframes; f0 += kBatch * kOrderThreads) {
        uint32_t c[kBatch];
        float e[kBatch];
        load(f0, c, e);
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
            const uint32_t f = f0 + u * kOrderThreads + t;
            if (f < nframes) order[cnt[bin(c[u], e[u])][t]++] = f;
        }
    }
}

__global__ void k_batched_status(const uint32_t *error, uint32_t *status) {
    if (threadIdx.x == 0) *status = *error;
}

using BatchedKernel = void (*)(BatchArgs);

template <typename T, int WPB, int NSMAX, bool STOP>
static BatchedKernel batched_kernel_w(int topo) {
    if (topo == kProduct) return k_batched<T, WPB, NSMAX, STOP, kProduct>;
    return k_batched<T, WPB, NSMAX, STOP, kGldpc>;
}

template <typename T, int NSMAX, bool STOP>
static BatchedKernel batched_kernel_n(int wpb, int topo) {
    if (wpb == 4) return batched_kernel_w<T, 4, NSMAX, STOP>(topo);
    if (wpb == 8) return batched_kernel_w<T, 8, NSMAX, STOP>(topo);
    return batched_kernel_w<T, 16, NSMAX, STOP>(topo);
}

// The instantiation for the batch: word width, the list-BLER stop (a separate
// instantiation, so that batches without it pay nothing), waves per group and topology.
template <typename T>
static BatchedKernel batched_kernel(int nmax, bool stop, int wpb, int topo) {
    if (nmax <= 32) return stop ? batched_kernel_n<T, 32, true>(wpb, topo) : batched_kernel_n<T, 32, false>(wpb, topo);
    if (nmax <= 64) return stop ? batched_kernel_n<T, 64, true>(wpb, topo) : batched_kernel_n<T, 64, false>(wpb, topo);
    return stop ? batched_kernel_n<T, 128, true>(wpb, topo) : batched_kernel_n<T, 128, false>(wpb, topo);
}

static int check_sched(const sogrand_sched_t *s) {
    if (s->waves_per_group != 4 && s->waves_per_group != 8 && s->waves_per_group != 16)
        return fail(SOGRAND_EINVAL, "waves_per_group must be 4, 8 or 16");
    if (s->frames_per_group < 1 || s->frames_per_group > kMaxSlots)
        return fail(SOGRAND_EINVAL, "frames_per_group outside 1..%d", kMaxSlots);
    if (s->steal_chunk < 1 || s->steal_chunk > SOGRAND_NMAX) return fail(SOGRAND_EINVAL, "steal_chunk outside 1..128");
    if (s->groups_per_cu < 1 || s->groups_per_cu > 64) return fail(SOGRAND_EINVAL, "groups_per_cu outside 1..64");
    return SOGRAND_OK;
}

// Tuned launch shapes by kind of batch: topology, precision, list-BLER stop on or off,
// and the (n, k) of its codes.
static std::mutex g_tuned_mu;
static std::map<std::string, sogrand_sched_t> g_tuned;

static std::string batch_kind(int topo, const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *p) {
    std::vector<std::pair<int, int>> nk;
    for (int i = 0; i < ncodes; i++) nk.emplace_back(codes[i]->n, codes[i]->k);
    std::sort(nk.begin(), nk.end());
    nk.erase(std::unique(nk.begin(), nk.end()), nk.end());
    std::string kind = topo == kProduct ? "product" : "gldpc";
    kind += p->precision == SOGRAND_F64 ? " f64" : " f32";
    kind += p->list_bler_stop > 0.0 ? " stop" : " nostop";
    for (const auto &c : nk) kind += " " + std::to_string(c.first) + ":" + std::to_string(c.second);
    return kind;
}

static int decode_batched(int topo, const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                          size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset,
                          uint64_t llr_len, const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                          uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                          uint32_t *status, const sogrand_sched_t *sched, void *stream) {
    SG_TRY(check_params(params));
    if (!codes || ncodes < 1 || ncodes > kMaxCodes) return fail(SOGRAND_EINVAL, "ncodes outside 1..%d", kMaxCodes);
    if (nframes == 0) return SOGRAND_OK;
    if (nframes >= (1ull << 31)) return fail(SOGRAND_EINVAL, "nframes too large");
    if (!frame_code || !frame_offset || !llr_ch || !hard || !success)
        return fail(SOGRAND_EINVAL, "frame_code, frame_offset, llr_ch, hard and success are required");
    for (int i = 0; i < ncodes; i++)
        if (!codes[i]) return fail(SOGRAND_EINVAL, "codes[%d] is NULL", i);
    sogrand_sched_t sc;
    sogrand_sched_default(&sc);
    bool chosen = sched != nullptr;
    if (sched) {
        sc = *sched;
    } else {
        std::lock_guard<std::mutex> g(g_tuned_mu);
        const auto it = g_tuned.find(batch_kind(topo, codes, ncodes, params));
        if (it != g_tuned.end()) {
            sc = it->second;
            chosen = true;
        }
    }
    SG_TRY(check_sched(&sc));
    BatchArgs a{};
    CodeTable table{};
    int nmax = 0;
    for (int i = 0; i < ncodes; i++) {
        SG_TRY(prepare_code(const_cast<sogrand_code_t *>(codes[i]), params->query_cap, &table.codes[i]));
        nmax = codes[i]->n > nmax ? codes[i]->n : nmax;
    }
    int dev = 0, cus = 0;
    SG_HIP(hipGetDevice(&dev));
    SG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (!chosen) {
        if (nframes <= (size_t)cus) {
            // a small batch: one frame per workgroup, of 16 waves, so that it spreads over as
            // many compute units as it has frames
            sc.waves_per_group = 16;
            sc.frames_per_group = 1;
            sc.steal_chunk = 2;
        } else if (nframes <= 8 * (size_t)cus) {
            sc.frames_per_group = 1;
        }
    }
    const bool f64 = params->precision == SOGRAND_F64;
    const BatchedKernel kern = f64 ? batched_kernel<double>(nmax, params->list_bler_stop > 0.0, sc.waves_per_group, topo)
                                   : batched_kernel<float>(nmax, params->list_bler_stop > 0.0, sc.waves_per_group, topo);
    const size_t dyn = sizeof(SlotLds) * sc.frames_per_group;
    // no more groups than fit on the compute units at once: a group that could not start
    // would find the frames taken when it did
    int resident = 0;
    SG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, reinterpret_cast<const void *>(kern),
                                                        kWave * sc.waves_per_group, dyn));
    if (resident < 1) return fail(SOGRAND_EINVAL, "launch shape does not fit a compute unit");
    const size_t per_cu = (size_t)(sc.groups_per_cu < resident ? sc.groups_per_cu : resident);
    const size_t want = (nframes + sc.frames_per_group - 1) / sc.frames_per_group;
    const size_t cap = (size_t)cus * per_cu;
    const int grid = (int)(want < cap ? want : cap);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    const size_t la_bytes = (size_t)grid * sc.frames_per_group * nmax * nmax * esz;
    char *ws = nullptr;
    // the frame order and each frame's ease, ahead of the code table
    const size_t order_bytes = (nframes * (sizeof(uint32_t) + sizeof(float)) + 511) & ~(size_t)255;
    const size_t head = 256 + ((sizeof(DevCode) * kMaxCodes + 255) & ~(size_t)255) + order_bytes;
    const size_t total = head + la_bytes;
    if (hipMallocAsync(reinterpret_cast<void **>(&ws), total, st) != hipSuccess)
        return fail(SOGRAND_ENOMEM, "work buffer allocation of %zu bytes failed", total);
    a.ncodes = ncodes;
    a.topo = topo;
    a.L = params->list_max;
    a.qcap = params->query_cap;
    a.pstop = params->list_bler_stop;
    a.alpha = params->alpha;
    a.max_iter = params->max_iter;
    a.early_stop = params->early_stop ? 1 : 0;
    a.nframes = (uint32_t)nframes;
    a.frame_code = frame_code;
    a.frame_offset = frame_offset;
    a.llr_len = llr_len;
    a.llr_ch = llr_ch;
    a.hard = hard;
    a.llr_app = llr_app;
    a.success = success;
    a.half_iters = half_iters;
    a.sumq = sum_queries;
    a.summax = sum_max_queries;
    a.codes = reinterpret_cast<const DevCode *>(ws + 256);
    a.la = ws + head;
    a.nmax = nmax;
    a.slots = sc.frames_per_group;
    a.chunk = sc.steal_chunk;
    a.next_frame = reinterpret_cast<uint32_t *>(ws);
    a.error = reinterpret_cast<uint32_t *>(ws) + 1;
    a.prof = prof_counters(PK_BATCHED);
    a.order = nullptr;
    hipLaunchKernelGGL(k_batched_init, dim3(1), dim3(64), 0, st, a.next_frame, table,
                       reinterpret_cast<DevCode *>(ws + 256), ncodes);
    {
        OrderKeys ok{};
        ok.ncodes = ncodes;
        ok.levels = kOrderBins - ncodes;
        int idx[kMaxCodes];
        for (int i = 0; i < ncodes; i++) idx[i] = i, ok.n[i] = codes[i]->n;
        std::stable_sort(idx, idx + ncodes, [&](int x, int y) { return codes[x]->n > codes[y]->n; });
        for (int r = 0; r < ncodes; r++) ok.rank[idx[r]] = (uint8_t)r;
        ok.last = idx[ncodes - 1];
        char *ob = ws + head - order_bytes;
        uint32_t *order = reinterpret_cast<uint32_t *>(ob);
        float *ease = reinterpret_cast<float *>(ob + ((nframes * sizeof(uint32_t) + 255) & ~(size_t)255));
        const dim3 eg((unsigned)((nframes + 3) / 4));
        if (f64)
            hipLaunchKernelGGL(k_frame_ease<double>, eg, dim3(256), 0, st, frame_code, frame_offset,
                               (uint32_t)nframes, llr_len, static_cast<const double *>(llr_ch), ok, ease);
        else
            hipLaunchKernelGGL(k_frame_ease<float>, eg, dim3(256), 0, st, frame_code, frame_offset,
                               (uint32_t)nframes, llr_len, static_cast<const float *>(llr_ch), ok, ease);
        hipLaunchKernelGGL(k_batched_order, dim3(1), dim3(kOrderThreads), 0, st, frame_code, ease,
                           (uint32_t)nframes, ok, order);
        a.order = order;
    }
    const int tok = prof_start(PK_BATCHED, st);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * sc.waves_per_group), dyn, st, a);
    prof_stop(tok, st);
    a.status = status;
    if (status) hipLaunchKernelGGL(k_batched_status, dim3(1), dim3(64), 0, st, a.error, status);
    int rc = SOGRAND_OK;
    if (hipGetLastError() != hipSuccess) rc = fail(SOGRAND_EDEVICE, "batched kernel launch failed");
    (void)hipFreeAsync(ws, st);
    return rc;
}

// Times one batched decode of the sample with shape s on st (the stream's work before
// it included).
static int time_shape(int topo, const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                      size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset, uint64_t llr_len,
                      const void *llr_ch, uint8_t *hard, uint8_t *success, const sogrand_sched_t &s,
                      hipEvent_t e0, hipEvent_t e1, hipStream_t st, float &ms) {
    SG_HIP(hipEventRecord(e0, st));
    SG_TRY(decode_batched(topo, codes, ncodes, params, nframes, frame_code, frame_offset, llr_len, llr_ch, hard,
                          nullptr, success, nullptr, nullptr, nullptr, nullptr, &s, st));
    SG_HIP(hipEventRecord(e1, st));
    SG_HIP(hipEventSynchronize(e1));
    SG_HIP(hipEventElapsedTime(&ms, e0, e1));
    return SOGRAND_OK;
}

static int tune(int topo, const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset, uint64_t llr_len,
                const void *llr_ch, sogrand_sched_t *best, float *best_ms, hipStream_t st) {
    if (!best) return fail(SOGRAND_EINVAL, "best is required");
    if (nframes == 0) return fail(SOGRAND_EINVAL, "the tuning sample is empty");
    SG_TRY(check_params(params));
    if (!codes || ncodes < 1 || ncodes > kMaxCodes) return fail(SOGRAND_EINVAL, "ncodes outside 1..%d", kMaxCodes);
    for (int i = 0; i < ncodes; i++)
        if (!codes[i]) return fail(SOGRAND_EINVAL, "codes[%d] is NULL", i);
    uint8_t *hard = nullptr, *success = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SOGRAND_OK;
    if (hipMalloc(reinterpret_cast<void **>(&hard), llr_len) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&success), nframes) != hipSuccess) {
        rc = fail(SOGRAND_ENOMEM, "tuning output buffers");
    } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = fail(SOGRAND_EDEVICE, "hipEventCreate failed");
    }
    sogrand_sched_t cur;
    sogrand_sched_default(&cur);
    float cur_ms = 0.f;
    // a shape's time: the better of two runs (the first run of all also builds the tables)
    auto measure = [&](const sogrand_sched_t &s, float &out) -> int {
        float t0 = 0.f, t1 = 0.f;
        SG_TRY(time_shape(topo, codes, ncodes, params, nframes, frame_code, frame_offset, llr_len, llr_ch, hard,
                          success, s, e0, e1, st, t0));
        SG_TRY(time_shape(topo, codes, ncodes, params, nframes, frame_code, frame_offset, llr_len, llr_ch, hard,
                          success, s, e0, e1, st, t1));
        out = t0 < t1 ? t0 : t1;
        return SOGRAND_OK;
    };
    if (rc == SOGRAND_OK) rc = measure(cur, cur_ms);
    static const int kWaves[] = {4, 8, 16}, kFrames[] = {1, 2, 3, 4}, kChunks[] = {1, 2, 4, 8};
    for (int field = 0; field < 3 && rc == SOGRAND_OK; field++) {
        const int *vals = field == 0 ? kWaves : field == 1 ? kFrames : kChunks;
        const int nv = field == 0 ? 3 : 4;
        const sogrand_sched_t base = cur;
        for (int j = 0; j < nv && rc == SOGRAND_OK; j++) {
            sogrand_sched_t cand = base;
            int &f = field == 0 ? cand.waves_per_group : field == 1 ? cand.frames_per_group : cand.steal_chunk;
            if (f == vals[j]) continue;
            f = vals[j];
            float t = 0.f;
            rc = measure(cand, t);
            if (rc == SOGRAND_OK && t < cur_ms) {
                cur = cand;
                cur_ms = t;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (hard) (void)hipFree(hard);
    if (success) (void)hipFree(success);
    if (rc != SOGRAND_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_tuned_mu);
        g_tuned[batch_kind(topo, codes, ncodes, params)] = cur;
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return SOGRAND_OK;
}

}  // namespace sg

extern "C" {

int sogrand_sched_tune(int gldpc, const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                       size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset, uint64_t llr_len,
                       const void *llr_ch, sogrand_sched_t *best, float *best_ms, void *stream) {
    return sg::tune(gldpc ? sg::kGldpc : sg::kProduct, codes, ncodes, params, nframes, frame_code, frame_offset,
                    llr_len, llr_ch, best, best_ms, static_cast<hipStream_t>(stream));
}

int sogrand_sched_table_save(const char *path) {
    if (!path) return sg::fail(SOGRAND_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> g(sg::g_tuned_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return sg::fail(SOGRAND_EINVAL, "cannot write %s", path);
    for (const auto &e : sg::g_tuned)
        std::fprintf(f, "%s|%d %d %d %d\n", e.first.c_str(), e.second.waves_per_group, e.second.frames_per_group,
                     e.second.steal_chunk, e.second.groups_per_cu);
    const bool ok = std::fclose(f) == 0;
    return ok ? SOGRAND_OK : sg::fail(SOGRAND_EINVAL, "cannot write %s", path);
}

int sogrand_sched_table_load(const char *path) {
    if (!path) return sg::fail(SOGRAND_EINVAL, "path is NULL");
    FILE *f = std::fopen(path, "r");
    if (!f) return sg::fail(SOGRAND_EINVAL, "cannot read %s", path);
    std::map<std::string, sogrand_sched_t> got;
    char line[512];
    int lineno = 0, rc = SOGRAND_OK;
    while (rc == SOGRAND_OK && std::fgets(line, sizeof line, f)) {
        lineno++;
        char *bar = std::strchr(line, '|');
        sogrand_sched_t s{};
        char tail = 0;
        if (!bar || bar == line ||
            std::sscanf(bar + 1, "%d %d %d %d %c", &s.waves_per_group, &s.frames_per_group, &s.steal_chunk,
                        &s.groups_per_cu, &tail) != 4 ||
            sg::check_sched(&s) != SOGRAND_OK) {
            rc = sg::fail(SOGRAND_EINVAL, "%s line %d: not a tuned shape", path, lineno);
            break;
        }
        got[std::string(line, bar)] = s;
    }
    std::fclose(f);
    if (rc != SOGRAND_OK) return rc;
    std::lock_guard<std::mutex> g(sg::g_tuned_mu);
    for (const auto &e : got) sg::g_tuned[e.first] = e.second;
    return (int)got.size();
}

void sogrand_sched_table_clear(void) {
    std::lock_guard<std::mutex> g(sg::g_tuned_mu);
    sg::g_tuned.clear();
}

void sogrand_sched_default(sogrand_sched_t *s) {
    if (!s) return;
    s->waves_per_group = 8;
    s->frames_per_group = 2;
    s->steal_chunk = 4;
    s->groups_per_cu = 8;
}

int sogrand_decode_batched(const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                           size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset,
                           uint64_t llr_len, const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                           uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                           uint32_t *status, const sogrand_sched_t *sched, void *stream) {
    return sg::decode_batched(sg::kProduct, codes, ncodes, params, nframes, frame_code, frame_offset, llr_len,
                              llr_ch, hard, llr_app, success, half_iters, sum_queries, sum_max_queries, status, sched,
                              stream);
}

int sogrand_decode_batched_gldpc(const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                                 size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset,
                                 uint64_t llr_len, const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                                 uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                                 uint32_t *status, const sogrand_sched_t *sched, void *stream) {
    return sg::decode_batched(sg::kGldpc, codes, ncodes, params, nframes, frame_code, frame_offset, llr_len,
                              llr_ch, hard, llr_app, success, half_iters, sum_queries, sum_max_queries, status, sched,
                              stream);
}

}  // extern "C"
