// Serving: continuous batching of product-frame decode requests.
//
// A host thread runs steps.  Each step advances every admitted frame by one
// half-iteration of the block turbo loop (section "Iterative decoding"): one
// wave per row or column, frames of every code in the same launches (one per
// word width), then one wave per frame tests the hard decision.  A frame that
// is valid (with early stopping) or has run its last half-iteration leaves:
// the check kernel writes its hard decision straight into pinned host memory
// and its slot is recycled.  Requests that arrived during a step join the next
// one, so the device is shared by frames at every stage of decoding.
//
// Frame state stays in a device slot for the frame's whole life.  Channel LLRs
// reach the device through pinned host memory that the first row pass reads
// directly (and copies into the slot), so admission costs no copy call.
//
// Several lanes (host threads, each with its own stream) run steps independently.
// A lane takes every request that arrived while its previous step ran, so a step
// held up by one long word delays only the frames of its own lane, and the other
// lanes' launches fill the device meanwhile.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

#include "word.hpp"

namespace sg {

constexpr int kServeCodes = 16;
constexpr size_t kServeMinBudget = (size_t)1 << 20;
// Independent step loops, each with its own stream and its own set of frames: while one
// lane's step waits for its slowest word, the others keep the device busy.
constexpr int kServeLanes = 4;

// One admitted frame in one step (device copy of the host's list).
struct ServeDesc {
    uint64_t slot;    // byte offset of the frame's slot, in both arenas
    uint32_t line0;   // first global line of this frame in its launch
    uint16_t code;    // index into the server's code table
    uint16_t n;
    uint32_t h;       // half-iteration run in this step, 1 .. 2 max_iter
    uint32_t pad;
};

// Written by the check kernel into pinned host memory, one per admitted frame.
struct ServeOut {
    uint32_t flags;   // bit 0: the hard decision is a product codeword; bit 1: the frame is finished
    uint32_t pad;
    uint64_t queries; // patterns tested in this step
};

// Byte layout of a frame's slot for code length n and element size esz, in device
// memory and in its pinned host copy alike: channel LLRs (carried in by the host copy),
// a-priori LLRs, the last pass's L_APP when the server exports it, the hard decision
// (carried out by the host copy) and the line masks.
struct SlotLayout {
    size_t la, app, hard, masks, bytes;
};

__host__ __device__ inline SlotLayout slot_layout(int n, size_t esz, bool app) {
    SlotLayout s;
    const size_t nn = (size_t)n * n;
    s.la = nn * esz;
    s.app = 2 * nn * esz;
    s.hard = s.app + (app ? nn * esz : 0);
    s.masks = (s.hard + nn + 15) & ~(size_t)15;
    s.bytes = (s.masks + (size_t)n * 2 * sizeof(uint64_t) + 255) & ~(size_t)255;
    return s;
}

struct ServeArgs {
    const DevCode *codes;
    char *arena;              // device slots
    const char *mirror;       // pinned host copy of the slots (device view)
    char *mirror_w;           // the same, for the check kernel's hard-decision export
    const ServeDesc *desc;    // this launch's frames
    uint32_t nact;            // frames in this launch
    uint32_t nlines;          // lines in this launch
    ServeOut *out;            // pinned host memory (device view), indexed like desc
    unsigned long long *qsum; // per frame: queries of this step
    int L;
    uint32_t qcap;
    double pstop;             // list-BLER stop threshold, 0 = off
    double alpha;
    int max_iter;
    int early_stop;
    int app;                  // keep each frame's L_APP and export it with the result
    ProfCounters *prof;
    // the pass launch covers the three word widths (32, 64, 128 bits): per width, its
    // frames' descriptors, counts and query sums, and its first workgroup
    const ServeDesc *wdesc[3];
    uint32_t wnact[3];
    uint32_t wlines[3];
    unsigned long long *wqsum[3];
    uint32_t wblock0[3];
};

// One wave per line: line gl of the launch's frames of one word width (a.desc, a.nact,
// a.nlines).  Every frame runs the half-iteration its descriptor names (rows for odd h).
template <typename T, int NS, bool STOP>
__device__ __forceinline__ void serve_line(const ServeArgs &a, uint32_t gl, WaveLds &S, int lane) {
    constexpr int NB = Lanes<NS>::NB;
    if (gl >= a.nlines) return;
    // the frame owning global line gl: the last descriptor whose line0 <= gl
    uint32_t lo = 0, hi = a.nact - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (load_uniform(&a.desc[mid].line0) <= gl) lo = mid;
        else hi = mid - 1;
    }
    const ServeDesc d = load_uniform(a.desc + lo);
    const DevCode *cdev = a.codes + d.code;
    const DevCode c = load_uniform(cdev);
    const int n = d.n;
    const int line = (int)(gl - d.line0);
    const SlotLayout sl = slot_layout(n, sizeof(T), a.app != 0);
    char *slot = a.arena + d.slot;
    T *ch = reinterpret_cast<T *>(slot);
    T *la = reinterpret_cast<T *>(slot + sl.la);
    T *app = reinterpret_cast<T *>(slot + sl.app);
    uint64_t *mk = reinterpret_cast<uint64_t *>(slot + sl.masks);
    const bool rows = (d.h & 1u) != 0;
    const T *src = reinterpret_cast<const T *>(a.mirror + d.slot);
    double lam[NB];
    int pos[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        pos[b] = rows ? line * n + i : i * n + line;
        lam[b] = 0.0;
        if (i < n) {
            if (d.h == 1) {
                // first half-iteration: the channel LLRs come from host memory and
                // stay in the slot; the a-priori LLRs are zero
                const T v = src[pos[b]];
                ch[pos[b]] = v;
                lam[b] = (double)v;
            } else {
                lam[b] = (double)ch[pos[b]] + (double)la[pos[b]];
            }
        }
    }
    double lapp[NB];
    const WordStats st = decode_word<NS, true, STOP>(c, cdev, a.L, a.qcap, a.pstop, lam, S, lapp, lane,
                                                     a.prof != nullptr);
    if (a.prof && lane == 0) prof_add(a.prof, st);
    uint64_t hm[2] = {0ull, 0ull};
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        const bool v = i < n;
        const bool neg = v && lapp[b] < 0.0;
        hm[b] = __ballot(neg);
        if (!v) continue;
        la[pos[b]] = (T)(a.alpha * (lapp[b] - lam[b]));
        if (a.app) app[pos[b]] = (T)lapp[b];
    }
    if (lane == 0) {
        mk[line * 2 + 0] = hm[0];
        mk[line * 2 + 1] = hm[1];
        atomicAdd(&a.qsum[lo], (unsigned long long)st.Q);
    }
}

// The pass of a step: one launch for all word widths, so that the lines of short codes run
// beside the long words of 128-bit ones instead of after them.  The 128-bit frames take the
// first workgroups, then the 64-bit ones, then the 32-bit ones.
template <typename T, bool STOP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_serve_pass(ServeArgs a) {
    __shared__ WaveLds lds[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const uint32_t b = blockIdx.x;
    const int w = b >= a.wblock0[0] ? 0 : (b >= a.wblock0[1] ? 1 : 2);
    ServeArgs g = a;
    g.desc = a.wdesc[w];
    g.nact = a.wnact[w];
    g.nlines = a.wlines[w];
    g.qsum = a.wqsum[w];
    const uint32_t gl = (b - a.wblock0[w]) * kWavesPerBlock + (uint32_t)wave;
    if (w == 2) serve_line<T, 128, STOP>(g, gl, lds[wave], lane);
    else if (w == 1) serve_line<T, 64, STOP>(g, gl, lds[wave], lane);
    else serve_line<T, 32, STOP>(g, gl, lds[wave], lane);
}

// OR of v over the wave, in every lane.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
    v |= xor_lane<1>(v);
    v |= xor_lane<2>(v);
    v |= xor_lane<4>(v);
    v |= xor_lane<8>(v);
    v |= xor_lane<16>(v);
    v |= xor_lane<32>(v);
    return v;
}

// One wave per frame of the step: validity of the hard decision (every line of
// the last pass and every cross line a codeword), the frame's outcome into host
// memory, and for a finished frame its hard decision (from the last pass's line
// masks: bit c of row j or bit j of column c is element [j][c]) and, when exported,
// its L_APP into the host copy.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_serve_check(ServeArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t i = (uint32_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (i >= a.nact) return;
    const ServeDesc d = load_uniform(a.desc + i);
    const int n = d.n;
    const SlotLayout sl = slot_layout(n, sizeof(T), a.app != 0);
    const char *slot = a.arena + d.slot;
    const uint64_t *mk = reinterpret_cast<const uint64_t *>(slot + sl.masks);
    const uint32_t *hcol = load_uniform(&a.codes[d.code].hcol);
    // The frame is a product codeword iff every line of the last pass and every line across
    // it has syndrome zero.  Bit-sliced over the parity bits p: with Hp the set of positions
    // whose H column has bit p, line x's syndrome bit p is the parity of (line x AND Hp), and
    // bit p of the cross lines' syndromes, as a vector over them, is the XOR of the lines l
    // in Hp.  Lane t holds lines t and t + 64 and the H columns of positions t and t + 64.
    __shared__ uint64_t mk_s[kWavesPerBlock][2 * SOGRAND_NMAX];
    const int wave = threadIdx.x / kWave;
    const bool v0 = lane < n, v1 = lane + kWave < n;
    const uint64_t a0 = v0 ? mk[lane * 2] : 0ull, a1 = v0 ? mk[lane * 2 + 1] : 0ull;
    const uint64_t b0 = v1 ? mk[(lane + kWave) * 2] : 0ull, b1 = v1 ? mk[(lane + kWave) * 2 + 1] : 0ull;
    const uint32_t h0 = v0 ? gptr(hcol)[lane] : 0u, h1 = v1 ? gptr(hcol)[lane + kWave] : 0u;
    if (v0) {
        mk_s[wave][lane * 2] = a0;
        mk_s[wave][lane * 2 + 1] = a1;
    }
    if (v1) {
        mk_s[wave][(lane + kWave) * 2] = b0;
        mk_s[wave][(lane + kWave) * 2 + 1] = b1;
    }
    const uint32_t used = __builtin_amdgcn_readfirstlane(wave_or(h0 | h1));   // the parity bits present
    bool bad = false;
    for (int p = 0; p < 32; p++) {
        if (!((used >> p) & 1u)) continue;
        const bool i0 = (h0 >> p) & 1u, i1 = (h1 >> p) & 1u;
        const uint64_t P0 = __ballot(i0), P1 = __ballot(i1);
        bad |= ((__popcll(a0 & P0) + __popcll(a1 & P1)) & 1) != 0;
        bad |= ((__popcll(b0 & P0) + __popcll(b1 & P1)) & 1) != 0;
        const uint64_t c0 = (i0 ? a0 : 0ull) ^ (i1 ? b0 : 0ull), c1 = (i0 ? a1 : 0ull) ^ (i1 ? b1 : 0ull);
        const uint32_t x = wave_xor((uint32_t)c0) | wave_xor((uint32_t)(c0 >> 32)) | wave_xor((uint32_t)c1) |
                           wave_xor((uint32_t)(c1 >> 32));
        bad |= x != 0u;
    }
    wave_sync();
    const bool valid = __ballot(bad) == 0ull;
    const bool finished = (valid && a.early_stop) || d.h == (uint32_t)(2 * a.max_iter);
    if (finished) {
        const bool rows = (d.h & 1u) != 0;
        uint8_t *hd = reinterpret_cast<uint8_t *>(a.mirror_w + d.slot + sl.hard);
        const int nn = n * n;
        // Whole 16-byte units per lane when a row of the frame is (n a multiple of 16): the
        // unit's 16 elements are 16 bits of one row of the hard decision, which the last pass's
        // masks give directly when its lines were rows, and their transpose (one ballot per row
        // and half) when they were columns.  Each 4 bits spread to 4 bytes with one multiply.
        // Otherwise 16-byte units that may straddle rows when n*n is a multiple of 16, else one
        // byte per lane.  The host copy is pinned host memory: 4-byte stores there
        // were seen to leave single bytes stale on the test machine, 16-byte stores never.
        if ((n & 15) == 0) {
            __shared__ uint64_t rm_s[kWavesPerBlock][2 * SOGRAND_NMAX];
            const uint64_t *rm = mk_s[wave];
            if (!rows) {
                for (int j = 0; j < n; j++) {
                    const int sh = j & 63;
                    const uint64_t ca = j < 64 ? a0 : a1, cb = j < 64 ? b0 : b1;   // columns lane, lane + 64
                    const uint64_t lo = __ballot((ca >> sh) & 1ull);
                    const uint64_t hi = __ballot((cb >> sh) & 1ull);
                    if (lane == 0) {
                        rm_s[wave][j * 2] = lo;
                        rm_s[wave][j * 2 + 1] = hi;
                    }
                }
                wave_sync();
                rm = rm_s[wave];
            }
            const int upr = n >> 4;   // 16-element units per row
            for (int u = lane; u < nn / 16; u += kWave) {
                const int j = u / upr, k = u - j * upr;
                const uint32_t b = (uint32_t)(rm[j * 2 + (k >> 2)] >> (16 * (k & 3))) & 0xffffu;
                uint32_t w[4];
                for (int q = 0; q < 4; q++) w[q] = (((b >> (4 * q)) & 0xfu) * 0x204081u) & 0x01010101u;
                *reinterpret_cast<uint4 *>(hd + 16 * u) = make_uint4(w[0], w[1], w[2], w[3]);
            }
        } else if ((nn & 15) == 0) {
            // 16-byte units that may straddle rows (n*n a multiple of 16: the unit is aligned)
            for (int o = lane * 16; o < nn; o += kWave * 16) {
                int j = o / n, c = o - j * n;
                uint32_t w[4];
                for (int q = 0; q < 4; q++) {
                    uint32_t v = 0;
                    for (int e = 0; e < 4; e++) {
                        const int line = rows ? j : c, bit = rows ? c : j;
                        v |= (uint32_t)((mk_s[wave][line * 2 + (bit >> 6)] >> (bit & 63)) & 1ull) << (8 * e);
                        if (++c == n) {
                            c = 0;
                            ++j;
                        }
                    }
                    w[q] = v;
                }
                *reinterpret_cast<uint4 *>(hd + o) = make_uint4(w[0], w[1], w[2], w[3]);
            }
        } else {
            for (int p = lane; p < nn; p += kWave) {
                const int j = p / n, c = p - j * n;
                const int line = rows ? j : c, bit = rows ? c : j;
                hd[p] = (uint8_t)((mk_s[wave][line * 2 + (bit >> 6)] >> (bit & 63)) & 1ull);
            }
        }
        if (a.app) {
            // 16-byte copies: n*n*sizeof(T) is a multiple of 16 when n is even, else 4-byte words
            const size_t bytes = (size_t)n * n * sizeof(T);
            const char *as = slot + sl.app;
            char *ad = a.mirror_w + d.slot + sl.app;
            if ((bytes & 15) == 0) {
                for (size_t o = (size_t)lane * 16; o < bytes; o += kWave * 16)
                    *reinterpret_cast<uint4 *>(ad + o) = *reinterpret_cast<const uint4 *>(as + o);
            } else {
                for (size_t o = (size_t)lane * 4; o < bytes; o += kWave * 4)
                    *reinterpret_cast<uint32_t *>(ad + o) = *reinterpret_cast<const uint32_t *>(as + o);
            }
        }
    }
    if (lane == 0) {
        ServeOut o;
        o.flags = (valid ? 1u : 0u) | (finished ? 2u : 0u);
        o.pad = 0;
        o.queries = a.qsum[i];
        a.out[i] = o;
        a.qsum[i] = 0ull;   // ready for the next step
    }
}

uint64_t clock_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

}  // namespace sg

using sg::ServeDesc;
using sg::ServeOut;

struct sogrand_server {
    struct Req {
        uint64_t id = 0, tag = 0;
        int code = 0, n = 0, wclass = 0;
        uint64_t slot = 0;
        uint32_t h = 1;
        uint64_t queries = 0;
        uint64_t t_submit = 0, t_admit = 0;
    };
    struct Done {
        sogrand_result_t r;
        std::vector<uint8_t> hard;
        std::vector<uint8_t> app;   // n*n LLRs in the server's precision, when exported
    };

    // one step loop: its thread, stream and per-step tables
    struct Lane {
        hipStream_t stream = nullptr;
        ServeDesc *desc_host = nullptr;      // pinned
        ServeDesc *desc_dev = nullptr;
        ServeOut *out_host = nullptr;        // pinned, written by the device
        ServeOut *out_dev = nullptr;         // device view of out_host
        unsigned long long *qsum = nullptr;  // device
        uint64_t last_step_end = 0;          // clock at the end of the previous step (0: idle)
        std::thread thread;
    };

    sogrand_params_t params{};
    int device = 0;
    size_t esz = 8;
    bool app = false;             // SOGRAND_SERVE_APP
    size_t budget = 0;
    char *arena = nullptr;        // device slots
    char *mirror = nullptr;       // pinned host copy (host pointer)
    char *mirror_dev = nullptr;   // the same (device pointer)
    size_t class_bytes[3] = {0, 0, 0};
    size_t bump = 0;
    std::vector<uint64_t> free_slots[3];
    size_t max_active = 0;

    const sogrand_code_t *code_ptr[sg::kServeCodes] = {};
    sg::DevCode *codes_host = nullptr;   // pinned staging of the table
    sg::DevCode *codes_dev = nullptr;
    int ncodes = 0;
    int ncodes_dev = 0;                  // table entries already on the device

    Lane lanes[sg::kServeLanes];

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> pending;
    std::deque<Done> done;
    size_t in_flight = 0;                // admitted, not yet finished
    uint64_t next_id = 1;
    bool stop = false;
    int error = SOGRAND_OK;
    sogrand_serve_stats_t stats{};

    void run(Lane &ln);
    int step(Lane &ln, std::vector<Req> &active);
    void release();
};

namespace sg {

static int width_class(int n) { return n <= 32 ? 0 : (n <= 64 ? 1 : 2); }
static int class_width(int c) { return c == 0 ? 32 : (c == 1 ? 64 : 128); }

template <typename T>
static void launch_serve_pass(const ServeArgs &a, uint32_t blocks, hipStream_t st) {
    if (a.pstop > 0.0) hipLaunchKernelGGL((k_serve_pass<T, true>), dim3(blocks), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_serve_pass<T, false>), dim3(blocks), dim3(kBlock), 0, st, a);
}

}  // namespace sg

// One step of lane `ln` over its admitted frames; updates `active` and publishes
// finished ones.
int sogrand_server::step(Lane &ln, std::vector<Req> &active) {
    using namespace sg;
    const uint64_t t0 = clock_ns();
    // frames grouped by word width, each group one launch
    std::vector<uint32_t> order;
    order.reserve(active.size());
    uint32_t gstart[4] = {0, 0, 0, 0};
    for (int c = 0; c < 3; c++) {
        gstart[c] = (uint32_t)order.size();
        for (uint32_t i = 0; i < active.size(); i++)
            if (active[i].wclass == c) order.push_back(i);
    }
    gstart[3] = (uint32_t)order.size();
    uint32_t glines[3] = {0, 0, 0};
    for (int c = 0; c < 3; c++) {
        for (uint32_t j = gstart[c]; j < gstart[c + 1]; j++) {
            const Req &r = active[order[j]];
            ServeDesc &d = ln.desc_host[j];
            d.slot = r.slot;
            d.line0 = glines[c];
            d.code = (uint16_t)r.code;
            d.n = (uint16_t)r.n;
            d.h = r.h;
            d.pad = 0;
            glines[c] += (uint32_t)r.n;
        }
    }
    const uint32_t nact = gstart[3];
    // host writes to the pinned arena (submitted LLRs) and the descriptor
    // staging complete before the device is told to read them
    std::atomic_thread_fence(std::memory_order_seq_cst);
    if (hipMemcpyAsync(ln.desc_dev, ln.desc_host, nact * sizeof(ServeDesc), hipMemcpyHostToDevice, ln.stream) !=
        hipSuccess)
        return fail(SOGRAND_EDEVICE, "descriptor copy failed");
    ServeArgs a{};
    a.codes = codes_dev;
    a.arena = arena;
    a.mirror = mirror_dev;
    a.mirror_w = mirror_dev;
    a.L = params.list_max;
    a.qcap = params.query_cap;
    a.pstop = params.list_bler_stop;
    a.alpha = params.alpha;
    a.max_iter = params.max_iter;
    a.early_stop = params.early_stop ? 1 : 0;
    a.app = app ? 1 : 0;
    a.prof = prof_counters(PK_SERVE);
    // one pass launch: the 128-bit frames' workgroups first, then the 64-bit and 32-bit ones
    uint32_t blocks = 0;
    for (int c = 2; c >= 0; c--) {
        a.wdesc[c] = ln.desc_dev + gstart[c];
        a.wnact[c] = gstart[c + 1] - gstart[c];
        a.wlines[c] = glines[c];
        a.wqsum[c] = ln.qsum + gstart[c];
        a.wblock0[c] = blocks;
        blocks += (glines[c] + kWavesPerBlock - 1) / kWavesPerBlock;
    }
    if (blocks) {
        if (esz == 8) launch_serve_pass<double>(a, blocks, ln.stream);
        else launch_serve_pass<float>(a, blocks, ln.stream);
    }
    ServeArgs ck = a;
    ck.desc = ln.desc_dev;
    ck.nact = nact;
    ck.out = ln.out_dev;
    ck.qsum = ln.qsum;
    const dim3 cg((nact + kWavesPerBlock - 1) / kWavesPerBlock);
    if (esz == 8) hipLaunchKernelGGL(k_serve_check<double>, cg, dim3(kBlock), 0, ln.stream, ck);
    else hipLaunchKernelGGL(k_serve_check<float>, cg, dim3(kBlock), 0, ln.stream, ck);
    if (hipGetLastError() != hipSuccess) return fail(SOGRAND_EDEVICE, "serving kernel launch failed");
    if (hipStreamSynchronize(ln.stream) != hipSuccess) return fail(SOGRAND_EDEVICE, "serving step failed on the device");
    const uint64_t t1 = clock_ns();

    std::vector<Done> fin;
    std::vector<Req> keep;
    keep.reserve(active.size());
    std::vector<uint8_t> is_done(active.size(), 0);
    for (uint32_t j = 0; j < nact; j++) {
        Req &r = active[order[j]];
        const ServeOut o = ln.out_host[j];
        r.queries += o.queries;
        if (o.flags & 2u) {
            Done dn;
            dn.r.request_id = r.id;
            dn.r.user_tag = r.tag;
            dn.r.status = SOGRAND_OK;
            dn.r.success = (uint8_t)(o.flags & 1u);
            dn.r.half_iters = (uint16_t)r.h;
            dn.r.n = (uint16_t)r.n;
            dn.r.queries = r.queries;
            dn.r.hard_offset = 0;
            dn.r.t_submit_ns = r.t_submit;
            dn.r.t_admit_ns = r.t_admit;
            dn.r.t_done_ns = t1;
            const SlotLayout sl = slot_layout(r.n, esz, app);
            const uint8_t *src = reinterpret_cast<const uint8_t *>(mirror + r.slot + sl.hard);
            dn.hard.assign(src, src + (size_t)r.n * r.n);
            if (app) {
                const uint8_t *as = reinterpret_cast<const uint8_t *>(mirror + r.slot + sl.app);
                dn.app.assign(as, as + (size_t)r.n * r.n * esz);
            }
            fin.push_back(std::move(dn));
            is_done[order[j]] = 1;
        } else {
            r.h += 1;
        }
    }
    for (uint32_t i = 0; i < active.size(); i++)
        if (!is_done[i]) keep.push_back(active[i]);
    {
        std::lock_guard<std::mutex> lk(mu);
        for (uint32_t i = 0; i < active.size(); i++)
            if (is_done[i]) free_slots[active[i].wclass].push_back(active[i].slot);
        for (Done &d : fin) done.push_back(std::move(d));
        in_flight -= fin.size();
        const double ms = (double)(t1 - t0) * 1e-6;
        stats.steps += 1;
        stats.frames += fin.size();
        stats.step_ms += ms;
        if (ms > stats.max_step_ms) stats.max_step_ms = ms;
        if (nact > stats.max_active) stats.max_active = nact;
        if (ln.last_step_end) stats.host_ms += (double)(t0 - ln.last_step_end) * 1e-6;
        ln.last_step_end = keep.empty() ? 0 : clock_ns();
    }
    active.swap(keep);
    if (!fin.empty()) cv_done.notify_all();
    return SOGRAND_OK;
}

void sogrand_server::run(Lane &ln) {
    using namespace sg;
    (void)hipSetDevice(device);
    std::vector<Req> active;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
            if (pending.empty() && active.empty()) break;   // stop requested and drained
            const uint64_t now = clock_ns();
            while (!pending.empty()) {
                Req r = pending.front();
                pending.pop_front();
                r.t_admit = now;
                active.push_back(r);
            }
            // codes registered since the last copy: only the new entries are written,
            // since other lanes' kernels may be reading the table
            if (ncodes > ncodes_dev && error == SOGRAND_OK) {
                const size_t off = (size_t)ncodes_dev, cnt = (size_t)(ncodes - ncodes_dev);
                if (hipMemcpyAsync(codes_dev + off, codes_host + off, sizeof(DevCode) * cnt, hipMemcpyHostToDevice,
                                   ln.stream) != hipSuccess ||
                    hipStreamSynchronize(ln.stream) != hipSuccess)
                    error = SOGRAND_EDEVICE;
                else
                    ncodes_dev = ncodes;
            }
        }
        int rc = error == SOGRAND_OK ? step(ln, active) : error;
        if (rc != SOGRAND_OK) {
            // the device failed: every request of this lane ends with the error
            std::lock_guard<std::mutex> lk(mu);
            error = rc;
            const uint64_t now = clock_ns();
            for (const Req &r : active) {
                Done dn;
                std::memset(&dn.r, 0, sizeof dn.r);
                dn.r.request_id = r.id;
                dn.r.user_tag = r.tag;
                dn.r.status = rc;
                dn.r.n = (uint16_t)r.n;
                dn.r.t_submit_ns = r.t_submit;
                dn.r.t_admit_ns = r.t_admit;
                dn.r.t_done_ns = now;
                done.push_back(std::move(dn));
                free_slots[r.wclass].push_back(r.slot);
            }
            in_flight -= active.size();
            active.clear();
            cv_done.notify_all();
        }
    }
}

// Frees every device and host resource (threads already joined).
void sogrand_server::release() {
    for (Lane &ln : lanes) {
        if (ln.stream) {
            (void)hipStreamSynchronize(ln.stream);
            (void)hipStreamDestroy(ln.stream);
        }
        if (ln.desc_host) (void)hipHostFree(ln.desc_host);
        if (ln.desc_dev) (void)hipFree(ln.desc_dev);
        if (ln.out_host) (void)hipHostFree(ln.out_host);
        if (ln.qsum) (void)hipFree(ln.qsum);
    }
    if (arena) (void)hipFree(arena);
    if (mirror) (void)hipHostFree(mirror);
    if (codes_host) (void)hipHostFree(codes_host);
    if (codes_dev) (void)hipFree(codes_dev);
}

extern "C" {

uint64_t sogrand_clock_ns(void) { return sg::clock_ns(); }

int sogrand_serve_create(const sogrand_params_t *params, size_t hbm_budget_bytes, unsigned flags,
                         sogrand_server_t **out) {
    using namespace sg;
    if (!out) return fail(SOGRAND_EINVAL, "out is NULL");
    *out = nullptr;
    SG_TRY(check_params(params));
    if (hbm_budget_bytes < kServeMinBudget) return fail(SOGRAND_EINVAL, "hbm_budget_bytes below 1 MiB");
    if (flags & ~(unsigned)SOGRAND_SERVE_APP) return fail(SOGRAND_EINVAL, "unknown flags 0x%x", flags);
    sogrand_server_t *s = new (std::nothrow) sogrand_server_t();
    if (!s) return fail(SOGRAND_ENOMEM, "server allocation failed");
    s->params = *params;
    s->esz = params->precision == SOGRAND_F64 ? 8 : 4;
    s->app = (flags & SOGRAND_SERVE_APP) != 0;
    s->budget = hbm_budget_bytes & ~(size_t)255;
    for (int c = 0; c < 3; c++) s->class_bytes[c] = slot_layout(class_width(c), s->esz, s->app).bytes;
    s->max_active = s->budget / s->class_bytes[0] + 1;
    auto cleanup = [s](int rc) {
        s->release();
        delete s;
        return rc;
    };
    if (hipGetDevice(&s->device) != hipSuccess) return cleanup(fail(SOGRAND_EDEVICE, "no current device"));
    if (hipMalloc(reinterpret_cast<void **>(&s->arena), s->budget) != hipSuccess)
        return cleanup(fail(SOGRAND_ENOMEM, "slot arena of %zu bytes", s->budget));
    // the device reads submitted LLRs from, and writes hard decisions and outcomes
    // to, these host allocations inside kernels: coherent and mapped
    const unsigned shared_flags = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc(reinterpret_cast<void **>(&s->mirror), s->budget, shared_flags) != hipSuccess)
        return cleanup(fail(SOGRAND_ENOMEM, "pinned host arena of %zu bytes", s->budget));
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&s->mirror_dev), s->mirror, 0) != hipSuccess)
        return cleanup(fail(SOGRAND_EDEVICE, "pinned host arena not visible to the device"));
    if (hipHostMalloc(reinterpret_cast<void **>(&s->codes_host), sizeof(DevCode) * kServeCodes, hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&s->codes_dev), sizeof(DevCode) * kServeCodes) != hipSuccess)
        return cleanup(fail(SOGRAND_ENOMEM, "server code table"));
    std::memset(s->codes_host, 0, sizeof(DevCode) * kServeCodes);
    for (sogrand_server::Lane &ln : s->lanes) {
        if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(SOGRAND_EDEVICE, "stream creation failed"));
        if (hipHostMalloc(reinterpret_cast<void **>(&ln.desc_host), sizeof(ServeDesc) * s->max_active,
                          hipHostMallocDefault) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&ln.desc_dev), sizeof(ServeDesc) * s->max_active) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&ln.out_host), sizeof(ServeOut) * s->max_active, shared_flags) !=
                hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&ln.qsum), sizeof(unsigned long long) * s->max_active) != hipSuccess)
            return cleanup(fail(SOGRAND_ENOMEM, "server tables"));
        if (hipHostGetDevicePointer(reinterpret_cast<void **>(&ln.out_dev), ln.out_host, 0) != hipSuccess)
            return cleanup(fail(SOGRAND_EDEVICE, "pinned result table not visible to the device"));
        if (hipMemsetAsync(ln.qsum, 0, sizeof(unsigned long long) * s->max_active, ln.stream) != hipSuccess ||
            hipStreamSynchronize(ln.stream) != hipSuccess)
            return cleanup(fail(SOGRAND_EDEVICE, "server initialisation failed"));
    }
    int started = 0;
    try {
        for (sogrand_server::Lane &ln : s->lanes) {
            ln.thread = std::thread([s, &ln] { s->run(ln); });
            started++;
        }
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        for (int i = 0; i < started; i++) s->lanes[i].thread.join();
        return cleanup(fail(SOGRAND_ENOMEM, "server thread could not start"));
    }
    *out = s;
    return SOGRAND_OK;
}

int sogrand_serve_submit(sogrand_server_t *s, const sogrand_code_t *code, const void *llr_ch_host, uint64_t user_tag,
                         uint64_t *request_id) {
    using namespace sg;
    if (!s || !code || !llr_ch_host) return fail(SOGRAND_EINVAL, "server, code and llr_ch_host are required");
    const int n = code->n;
    const int wc = width_class(n);
    sogrand_server::Req r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->error != SOGRAND_OK) return fail(s->error, "the server's device failed");
        if (s->stop) return fail(SOGRAND_EINVAL, "server is shutting down");
        int ci = -1;
        for (int i = 0; i < s->ncodes; i++)
            if (s->code_ptr[i] == code) ci = i;
        if (ci < 0) {
            if (s->ncodes == kServeCodes) return fail(SOGRAND_EINVAL, "a server accepts at most %d codes", kServeCodes);
            // the code's tables are built on the server's device; the caller's
            // current device is restored afterwards
            DevCode dc;
            int prev = 0;
            if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(s->device) != hipSuccess)
                return fail(SOGRAND_EDEVICE, "cannot select the server's device");
            const int rc = prepare_code(const_cast<sogrand_code_t *>(code), s->params.query_cap, &dc);
            (void)hipSetDevice(prev);
            if (rc != SOGRAND_OK) return rc;
            ci = s->ncodes++;
            s->code_ptr[ci] = code;
            s->codes_host[ci] = dc;
        }
        // a slot: a recycled one of this width, else fresh space in the arena
        if (!s->free_slots[wc].empty()) {
            r.slot = s->free_slots[wc].back();
            s->free_slots[wc].pop_back();
        } else if (s->bump + s->class_bytes[wc] <= s->budget) {
            r.slot = s->bump;
            s->bump += s->class_bytes[wc];
        } else {
            return SOGRAND_EAGAIN;
        }
        r.id = s->next_id++;
        r.code = ci;
    }
    // the slot is reserved: fill its host copy outside the lock
    std::memcpy(s->mirror + r.slot, llr_ch_host, (size_t)n * n * s->esz);
    r.tag = user_tag;
    r.n = n;
    r.wclass = wc;
    r.h = 1;
    r.t_submit = clock_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->pending.push_back(r);
        s->in_flight += 1;
    }
    s->cv_work.notify_one();
    if (request_id) *request_id = r.id;
    return SOGRAND_OK;
}

int sogrand_serve_poll(sogrand_server_t *s, sogrand_result_t *results, size_t max_results, size_t *n_results,
                       uint8_t *hard_out_host, void *llr_app_out_host, int64_t timeout_ns) {
    using namespace sg;
    if (!s || !results || !n_results || max_results == 0)
        return fail(SOGRAND_EINVAL, "server, results, n_results and max_results > 0 are required");
    *n_results = 0;
    // the finished frames are taken under the lock and copied out after it, so that the
    // lanes, which take the lock between steps, never wait on the caller's copies
    std::vector<sogrand_server::Done> got;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->done.empty()) {
            if (s->in_flight == 0) return SOGRAND_ENOTFOUND;
            if (timeout_ns == 0) return SOGRAND_ETIMEDOUT;
            auto ready = [&] { return !s->done.empty() || s->in_flight == 0; };
            if (timeout_ns < 0) s->cv_done.wait(lk, ready);
            else s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready);
            if (s->done.empty()) return s->in_flight == 0 ? SOGRAND_ENOTFOUND : SOGRAND_ETIMEDOUT;
        }
        const size_t k = s->done.size() < max_results ? s->done.size() : max_results;
        got.reserve(k);
        for (size_t i = 0; i < k; i++) {
            got.push_back(std::move(s->done.front()));
            s->done.pop_front();
        }
    }
    size_t off = 0;
    for (size_t k = 0; k < got.size(); k++) {
        const sogrand_server::Done &d = got[k];
        results[k] = d.r;
        results[k].hard_offset = off;
        if (hard_out_host && !d.hard.empty()) std::memcpy(hard_out_host + off, d.hard.data(), d.hard.size());
        if (llr_app_out_host && !d.app.empty())
            std::memcpy(static_cast<char *>(llr_app_out_host) + off * s->esz, d.app.data(), d.app.size());
        off += (size_t)d.r.n * d.r.n;
    }
    *n_results = got.size();
    return SOGRAND_OK;
}

int sogrand_serve_replay(sogrand_server_t *s, const sogrand_code_t *const *codes, int ncodes, size_t nreq,
                         const uint8_t *req_code, const uint64_t *req_offset, const void *llr_host,
                         uint64_t llr_len, const uint64_t *arrival_ns, uint64_t t0_ns, uint64_t *retries) {
    using namespace sg;
    if (!s || !codes || ncodes < 1 || (nreq && (!req_code || !req_offset || !llr_host || !arrival_ns)))
        return fail(SOGRAND_EINVAL, "server, codes, and the request arrays are required");
    for (int i = 0; i < ncodes; i++)
        if (!codes[i]) return fail(SOGRAND_EINVAL, "codes[%d] is NULL", i);
    const char *base = static_cast<const char *>(llr_host);
    uint64_t again = 0;
    for (size_t i = 0; i < nreq; i++) {
        if (req_code[i] >= ncodes) return fail(SOGRAND_EINVAL, "request %zu: code index out of range", i);
        const uint64_t nn = (uint64_t)codes[req_code[i]]->n * codes[req_code[i]]->n;
        if (req_offset[i] > llr_len || llr_len - req_offset[i] < nn)
            return fail(SOGRAND_EINVAL, "request %zu: LLRs outside llr_host", i);
        const uint64_t due = t0_ns + arrival_ns[i];
        while (clock_ns() < due) {
        }
        for (;;) {
            const int rc = sogrand_serve_submit(s, codes[req_code[i]], base + req_offset[i] * s->esz, i, nullptr);
            if (rc == SOGRAND_OK) break;
            if (rc != SOGRAND_EAGAIN) return rc;
            again++;
            std::this_thread::yield();
        }
    }
    if (retries) *retries = again;
    return SOGRAND_OK;
}

int sogrand_serve_stats(sogrand_server_t *s, sogrand_serve_stats_t *stats) {
    if (!s || !stats) return sg::fail(SOGRAND_EINVAL, "server and stats are required");
    std::lock_guard<std::mutex> lk(s->mu);
    *stats = s->stats;
    return SOGRAND_OK;
}

int sogrand_serve_destroy(sogrand_server_t *s) {
    if (!s) return SOGRAND_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (sogrand_server::Lane &ln : s->lanes)
        if (ln.thread.joinable()) ln.thread.join();
    (void)hipSetDevice(s->device);
    s->release();
    delete s;
    return SOGRAND_OK;
}

}  // extern "C"
