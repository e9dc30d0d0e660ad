// Internal declarations of libsogrand (not installed; the public API is include/sogrand.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sogrand.h"

namespace sg {

// ----------------------------------------------------------------------------
// errors
// ----------------------------------------------------------------------------
int fail(int code, const char *fmt, ...);

#define SG_HIP(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::sg::fail(SOGRAND_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define SG_TRY(expr)                \
    do {                            \
        int rc_ = (expr);           \
        if (rc_ != SOGRAND_OK) return rc_; \
    } while (0)

// ----------------------------------------------------------------------------
// query schedule: the ORBGRAND order in rank space, shared by every word of a code
// ----------------------------------------------------------------------------
// Pattern t of parity class c is pat[c][t]: up to 16 ranks (1..n) as bytes,
// ascending, zero padded.  wmax[c][t/64] is the largest Hamming weight among
// patterns 64*(t/64) .. 64*(t/64)+63.  Even codes have two classes (even and
// odd weights); other codes one class holding every weight.
struct Schedule {
    int device = -1;
    uint32_t cap = 0;         // patterns requested per class
    uint32_t len[2] = {0, 0}; // patterns stored per class (< cap only if the class is exhausted)
    uint4 *pat[2] = {nullptr, nullptr};
    uint32_t *wmax[2] = {nullptr, nullptr};
};

// Frame topology: a product code (rows and columns) or a QC-GLDPC code (two block
// rows of circulants); which variable nodes form each component word is described
// where the kernels map words to frame positions.
constexpr int kProduct = 0, kGldpc = 1;
// zero patterns after the end of each query schedule: two 64-pattern chunks
constexpr size_t kSchedPad = 128;

// Device-side view of a code and its schedule, passed by value to kernels.
struct DevCode {
    const uint32_t *hcol;   // [n] parity-check column of each bit
    const uint4 *pat[2];
    const uint32_t *wmax[2];
    uint32_t len[2];
    int n;
    int even;
    double phi;             // random-codebook hit probability used by Corollary 1
};

}  // namespace sg

struct sogrand_code {
    int n = 0, k = 0, r = 0, even = 0;
    uint32_t hcol[SOGRAND_NMAX] = {};
    double phi = 0.0;
    std::mutex mu;
    std::map<int, uint32_t *> d_hcol;                // per device
    std::map<int, sg::Schedule *> sched;             // per device: largest cap built so far
    std::vector<sg::Schedule *> retired;             // superseded schedules, freed at destroy
};

namespace sg {

// Ensures the device copy of H and a schedule covering query_cap on the current
// device, then fills *dc.  The first call for a (code, device, larger cap) builds
// the schedule and waits for it.  With may_allocate false nothing is built: a
// missing table is an EINVAL.
int prepare_code(sogrand_code_t *code, uint32_t query_cap, DevCode *dc, bool may_allocate = true);

int check_params(const sogrand_params_t *p);

// ----------------------------------------------------------------------------
// measurement hooks
// ----------------------------------------------------------------------------
enum ProfKind { PK_COMPONENT = 0, PK_PASS, PK_CHECK, PK_INIT, PK_BATCHED, PK_SERVE, PK_COUNT };

// Phases of a component decode timed by builds with SG_PHASE_CLOCKS (wave clock cycles):
// hard decision, syndrome and rho; ranking; class masses; query loop; soft output; the
// rest of the line's work in the kernel (reading the inputs, writing the outputs); and, in
// the persistent kernel, the time a wave spends finding work (claims and waiting) and the
// time spent on half-iteration hand-overs (validity check, retiring and refilling a slot).
constexpr int kPhases = 8;

struct ProfCounters {
    unsigned long long words, queries, ranks, exact_rank;   // exact_rank: words that needed the exact ranking pass
    unsigned long long phase[kPhases];                       // SG_PHASE_CLOCKS builds only
};
// Each kernel family owns kProfSlots counter slots; a workgroup adds to slot
// blockIdx.x % kProfSlots so that the atomics do not contend on one address.
constexpr int kProfSlots = 256;

// First of the kProfSlots device counters for `kind` while work counting is on, else nullptr.
ProfCounters *prof_counters(ProfKind kind);
// Returns an opaque token (or -1 when profiling is off) after recording a start event.
int prof_start(ProfKind kind, hipStream_t st);
void prof_stop(int token, hipStream_t st);

void free_schedule(Schedule *s);

}  // namespace sg
