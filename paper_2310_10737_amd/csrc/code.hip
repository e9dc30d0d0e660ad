// Codes, parameters, errors and the per-code query schedule of libsogrand.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.hpp"

namespace sg {

static thread_local std::string g_last_error = "no error";

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// ----------------------------------------------------------------------------
// GF(2) helpers on parity-check columns
// ----------------------------------------------------------------------------
// Rank of H and whether the all-ones word lies in its row space (then every
// codeword c satisfies 1.c = 0, i.e. has even weight: the code is "even").
static void h_rank_even(int n, int r, const uint32_t *hcol, int *rank, int *even) {
    // rows as 128-bit masks over the n columns
    uint64_t rows[32][2] = {};
    for (int j = 0; j < n; j++)
        for (int i = 0; i < r; i++)
            if ((hcol[j] >> i) & 1u) rows[i][j >> 6] |= 1ull << (j & 63);
    uint64_t ones[2] = {0, 0};
    for (int j = 0; j < n; j++) ones[j >> 6] |= 1ull << (j & 63);
    int rk = 0;
    int pivots[32];
    for (int col = 0; col < n && rk < r; col++) {
        int w = col >> 6;
        uint64_t bit = 1ull << (col & 63);
        int sel = -1;
        for (int i = rk; i < r; i++)
            if (rows[i][w] & bit) { sel = i; break; }
        if (sel < 0) continue;
        std::swap(rows[sel][0], rows[rk][0]);
        std::swap(rows[sel][1], rows[rk][1]);
        for (int i = 0; i < r; i++)
            if (i != rk && (rows[i][w] & bit)) { rows[i][0] ^= rows[rk][0]; rows[i][1] ^= rows[rk][1]; }
        pivots[rk++] = col;
    }
    for (int i = 0; i < rk; i++) {
        int col = pivots[i];
        if ((ones[col >> 6] >> (col & 63)) & 1ull) { ones[0] ^= rows[i][0]; ones[1] ^= rows[i][1]; }
    }
    *rank = rk;
    *even = (ones[0] | ones[1]) == 0;
}

static const uint32_t kPrimPoly[8] = {0, 0, 0, 0b1011, 0b10011, 0b100101, 0b1000011, 0b10001001};

// Extended BCH parity-check columns: for the cyclic code of length 2^m - 1 with
// zeros alpha^1, alpha^3, ..., alpha^(2t-1), column j < n-1 stacks the m-bit
// field elements alpha^{(2i-1) j} (i = 1..t) and a final 1 for the overall parity
// row; column n-1 is the overall parity row alone.  Redundant rows are dropped by
// the caller's rank check only when t = 1 is not enough; here t is chosen from k.
static int ebch_columns(int n, int k, uint32_t *hcol) {
    int m = 0;
    while ((1 << m) < n) m++;
    if ((1 << m) != n || m < 3 || m > 7) return fail(SOGRAND_EINVAL, "eBCH length %d not supported", n);
    const int nc = n - 1;
    int t;
    if (k == n - 1 - m) t = 1;
    else if (n == 16 && k == 7) t = 2;
    else return fail(SOGRAND_EINVAL, "eBCH [%d,%d] not supported", n, k);
    // powers of alpha in the polynomial basis
    uint32_t ex[128];
    uint32_t x = 1;
    for (int i = 0; i < nc; i++) {
        ex[i] = x;
        x <<= 1;
        if (x & (1u << m)) x ^= kPrimPoly[m];
    }
    int rows = t * m + 1;
    for (int j = 0; j < n; j++) {
        uint32_t c = 0;
        if (j < nc) {
            for (int i = 0; i < t; i++) c |= ex[((2 * i + 1) * j) % nc] << (i * m);
        }
        c |= 1u << (rows - 1);
        hcol[j] = c;
    }
    return rows;
}

// Reduce an H with possibly dependent rows (given as `rows` bit planes of hcol) to
// a full-rank basis of the same row space with n-k rows.
static int reduce_rows(int n, int rows, uint32_t *hcol, int want) {
    uint64_t R[32][2] = {};
    for (int j = 0; j < n; j++)
        for (int i = 0; i < rows; i++)
            if ((hcol[j] >> i) & 1u) R[i][j >> 6] |= 1ull << (j & 63);
    uint64_t B[32][2];
    int nb = 0;
    for (int i = 0; i < rows; i++) {
        uint64_t v0 = R[i][0], v1 = R[i][1];
        for (int b = 0; b < nb; b++) {
            // pivot of basis row b = its highest set bit
            int piv = B[b][1] ? 64 + 63 - __builtin_clzll(B[b][1]) : 63 - __builtin_clzll(B[b][0]);
            uint64_t bit = piv >= 64 ? (v1 >> (piv - 64)) & 1ull : (v0 >> piv) & 1ull;
            if (bit) { v0 ^= B[b][0]; v1 ^= B[b][1]; }
        }
        if (v0 | v1) { B[nb][0] = v0; B[nb][1] = v1; nb++; }
    }
    if (nb != want) return fail(SOGRAND_EINVAL, "parity-check rank %d, expected %d", nb, want);
    for (int j = 0; j < n; j++) {
        uint32_t c = 0;
        for (int b = 0; b < nb; b++)
            if ((B[b][j >> 6] >> (j & 63)) & 1ull) c |= 1u << b;
        hcol[j] = c;
    }
    return SOGRAND_OK;
}

static double hit_probability(int n, int k, int even) {
    // (2^k - 1) / (2^N - 1) with N = n - 1 inside one parity class of an even code
    long double num = ldexpl(1.0L, k) - 1.0L;
    long double den = ldexpl(1.0L, even ? n - 1 : n) - 1.0L;
    return (double)(num / den);
}

static int make_code(int n, int k, const uint32_t *hcol, sogrand_code_t **out) {
    int rank = 0, even = 0;
    h_rank_even(n, n - k, hcol, &rank, &even);
    if (rank != n - k) return fail(SOGRAND_EINVAL, "H has rank %d, expected n-k = %d", rank, n - k);
    auto *c = new (std::nothrow) sogrand_code();
    if (!c) return fail(SOGRAND_ENOMEM, "out of host memory");
    c->n = n;
    c->k = k;
    c->r = n - k;
    c->even = even;
    std::memcpy(c->hcol, hcol, sizeof(uint32_t) * n);
    c->phi = hit_probability(n, k, even);
    *out = c;
    return SOGRAND_OK;
}

int check_params(const sogrand_params_t *p) {
    if (!p) return fail(SOGRAND_EINVAL, "params is NULL");
    if (p->list_max < 1 || p->list_max > SOGRAND_LIST_MAX)
        return fail(SOGRAND_EINVAL, "list_max %d outside 1..%d", p->list_max, SOGRAND_LIST_MAX);
    if (p->query_cap < 1 || p->query_cap > SOGRAND_QUERY_CAP_MAX)
        return fail(SOGRAND_EINVAL, "query_cap %u outside 1..2^24", p->query_cap);
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(SOGRAND_EINVAL, "alpha must be finite and > 0");
    if (p->max_iter < 1 || p->max_iter > 1000) return fail(SOGRAND_EINVAL, "max_iter %d outside 1..1000", p->max_iter);
    if (p->precision != SOGRAND_F64 && p->precision != SOGRAND_F32)
        return fail(SOGRAND_EINVAL, "precision must be SOGRAND_F64 or SOGRAND_F32");
    if (!(p->list_bler_stop >= 0.0 && p->list_bler_stop <= 1.0))
        return fail(SOGRAND_EINVAL, "list_bler_stop must lie in [0, 1]");
    return SOGRAND_OK;
}

// ----------------------------------------------------------------------------
// schedule construction
// ----------------------------------------------------------------------------
struct ClassDesc {
    uint32_t off, cnt;   // first pattern index and number of patterns to write
    uint16_t W;          // logistic weight
    uint8_t w;           // Hamming weight
    uint8_t pad;
};

// Lexicographically smallest strictly increasing parts u[from..w-1], each > prev
// and <= n, summing to T (a completion is known to exist).  Greedy from the left:
// each part is as small as the parts after it (at most the largest values <= n)
// allow.
__device__ static void fill_tail(uint8_t *u, int from, int w, int prev, int T, int n) {
    for (int j = from; j < w; j++) {
        int r = w - 1 - j;
        int maxrest = r * n - r * (r - 1) / 2;
        int x = prev + 1 > T - maxrest ? prev + 1 : T - maxrest;
        u[j] = (uint8_t)x;
        T -= x;
        prev = x;
    }
}

// Successor in lexicographic order among distinct-part partitions of W into w
// parts <= n.  In the coordinates v_j = u_j - j (non-decreasing) this is the
// landslide move: raise the rightmost position that can still be raised and let
// the remaining mass settle as flat as possible towards the left.
__device__ static bool next_tuple(uint8_t *u, int w, int W, int n) {
    int prefix[16];
    int s = 0;
    for (int j = 0; j < w; j++) { prefix[j] = s; s += u[j]; }
    for (int i = w - 2; i >= 0; i--) {
        int nv = u[i] + 1;
        int m = w - 1 - i;
        int T = W - prefix[i] - nv;
        int minsum = m * (nv + 1) + m * (m - 1) / 2;
        int maxsum = m * n - m * (m - 1) / 2;
        if (T >= minsum && T <= maxsum) {
            u[i] = (uint8_t)nv;
            fill_tail(u, i + 1, w, nv, T, n);
            return true;
        }
    }
    return false;
}

__device__ static uint4 pack16(const uint8_t *u, int w) {
    uint32_t d[4] = {0, 0, 0, 0};
    for (int j = 0; j < w; j++) d[j >> 2] |= (uint32_t)u[j] << (8 * (j & 3));
    return make_uint4(d[0], d[1], d[2], d[3]);
}

// One thread per (W, w) class writes that class's patterns in order.
__global__ void k_schedule(const ClassDesc *cls, int ncls, int n, uint4 *pat) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncls) return;
    ClassDesc d = cls[c];
    uint8_t u[16];
    if (d.w == 0) {
        pat[d.off] = make_uint4(0, 0, 0, 0);
        return;
    }
    fill_tail(u, 0, d.w, 0, d.W, n);
    for (uint32_t t = 0; t < d.cnt; t++) {
        pat[d.off + t] = pack16(u, d.w);
        if (t + 1 < d.cnt && !next_tuple(u, d.w, d.W, n)) break;
    }
}

static int build_schedule(const sogrand_code_t *c, int dev, uint32_t cap, Schedule **out) {
    const int n = c->n;
    const int Wlim = n * (n + 1) / 2 < 600 ? n * (n + 1) / 2 : 600;
    const int WMAXW = 16;
    // dp[w][W]: subsets of {1..n} with w elements summing to W (w <= 16), saturating
    std::vector<uint64_t> dp((WMAXW + 1) * (Wlim + 1), 0);
    auto at = [&](int w, int W) -> uint64_t & { return dp[(size_t)w * (Wlim + 1) + W]; };
    const uint64_t SAT = 1ull << 62;
    at(0, 0) = 1;
    for (int i = 1; i <= n; i++)
        for (int w = (i < WMAXW ? i : WMAXW); w >= 1; w--)
            for (int W = Wlim; W >= i; W--) {
                uint64_t v = at(w, W) + at(w - 1, W - i);
                at(w, W) = v > SAT ? SAT : v;
            }

    auto *s = new (std::nothrow) Schedule();
    if (!s) return fail(SOGRAND_ENOMEM, "out of host memory");
    s->device = dev;
    s->cap = cap;
    const int ncls = c->even ? 2 : 1;
    std::vector<ClassDesc> descs[2];
    std::vector<uint32_t> wmax[2];
    for (int cl = 0; cl < ncls; cl++) {
        uint64_t off = 0;
        // patterns with more than 16 parts cannot be stored; in this class the first
        // such pattern has 17 (odd) or 18 (even) parts and logistic weight >= 153 or 171
        const int wide = (c->even && cl == 0) ? 18 : 17;
        const int wide_W = wide * (wide + 1) / 2;
        for (int W = 0; W <= Wlim && off < cap; W++) {
            if (n >= wide && W >= wide_W) {
                delete s;
                return fail(SOGRAND_EINVAL, "query cap %u reaches patterns of weight > 16 for n = %d", cap, n);
            }
            for (int w = 0; w <= WMAXW && w <= n && off < cap; w++) {
                if (c->even && (w & 1) != cl) continue;
                uint64_t cnt = at(w, W);
                if (!cnt) continue;
                uint64_t take = cnt < cap - off ? cnt : cap - off;
                descs[cl].push_back(ClassDesc{(uint32_t)off, (uint32_t)take, (uint16_t)W, (uint8_t)w, 0});
                off += take;
            }
        }
        s->len[cl] = (uint32_t)off;
        size_t nch = (off + 63) / 64;
        wmax[cl].assign(nch ? nch : 1, 0);
        for (const ClassDesc &d : descs[cl]) {
            if (!d.cnt) continue;
            for (size_t ch = d.off / 64; ch <= (d.off + d.cnt - 1) / 64; ch++)
                if (wmax[cl][ch] < d.w) wmax[cl][ch] = d.w;
        }
    }

    hipStream_t st;
    SG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    int rc = SOGRAND_OK;
    ClassDesc *d_desc = nullptr;
    for (int cl = 0; cl < ncls && rc == SOGRAND_OK; cl++) {
        // the patterns, then two chunks of zero patterns: the decode loads whole 64-pattern
        // chunks up to two past the one it tests, without per-lane bounds
        const size_t npat = s->len[cl] + kSchedPad;
        if (hipMalloc(&s->pat[cl], npat * sizeof(uint4)) != hipSuccess ||
            hipMalloc(&s->wmax[cl], wmax[cl].size() * sizeof(uint32_t)) != hipSuccess) {
            rc = fail(SOGRAND_ENOMEM, "device allocation of the query schedule failed");
            break;
        }
        if (hipMemcpyAsync(s->wmax[cl], wmax[cl].data(), wmax[cl].size() * sizeof(uint32_t), hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = fail(SOGRAND_EDEVICE, "copy of the schedule weights failed");
            break;
        }
        size_t nd = descs[cl].size();
        if (!nd) continue;
        if (hipMalloc(&d_desc, nd * sizeof(ClassDesc)) != hipSuccess) {
            rc = fail(SOGRAND_ENOMEM, "device allocation failed");
            break;
        }
        if (hipMemcpyAsync(d_desc, descs[cl].data(), nd * sizeof(ClassDesc), hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = fail(SOGRAND_EDEVICE, "copy of the schedule classes failed");
            break;
        }
        if (hipMemsetAsync(s->pat[cl] + s->len[cl], 0, kSchedPad * sizeof(uint4), st) != hipSuccess) {
            rc = fail(SOGRAND_EDEVICE, "clearing the schedule's padding failed");
            break;
        }
        hipLaunchKernelGGL(k_schedule, dim3((unsigned)((nd + 63) / 64)), dim3(64), 0, st, d_desc, (int)nd, n, s->pat[cl]);
        if (hipGetLastError() != hipSuccess) {
            rc = fail(SOGRAND_EDEVICE, "schedule kernel launch failed");
            break;
        }
        if (hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(SOGRAND_EDEVICE, "schedule build failed");
            break;
        }
        (void)hipFree(d_desc);
        d_desc = nullptr;
    }
    if (d_desc) (void)hipFree(d_desc);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (rc != SOGRAND_OK) {
        free_schedule(s);
        return rc;
    }
    *out = s;
    return SOGRAND_OK;
}

void free_schedule(Schedule *s) {
    if (!s) return;
    for (int c = 0; c < 2; c++) {
        if (s->pat[c]) (void)hipFree(s->pat[c]);
        if (s->wmax[c]) (void)hipFree(s->wmax[c]);
    }
    delete s;
}

int prepare_code(sogrand_code_t *code, uint32_t query_cap, DevCode *dc, bool may_allocate) {
    if (!code) return fail(SOGRAND_EINVAL, "code is NULL");
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(code->mu);
    if (!may_allocate) {
        auto h = code->d_hcol.find(dev);
        auto t = code->sched.find(dev);
        if (h == code->d_hcol.end() || !h->second || t == code->sched.end() || !t->second ||
            t->second->cap < query_cap)
            return fail(SOGRAND_EINVAL,
                        "the code's tables for device %d and query cap %u are not built: decode once with this "
                        "code on this device with a cap at least this large first", dev, query_cap);
    }
    uint32_t *&hc = code->d_hcol[dev];
    if (!hc) {
        if (hipMalloc(&hc, sizeof(uint32_t) * SOGRAND_NMAX) != hipSuccess) {
            hc = nullptr;
            return fail(SOGRAND_ENOMEM, "device allocation failed");
        }
        SG_HIP(hipMemcpy(hc, code->hcol, sizeof(uint32_t) * SOGRAND_NMAX, hipMemcpyHostToDevice));
    }
    Schedule *&s = code->sched[dev];
    if (!s || s->cap < query_cap) {
        // grow geometrically so that nearby caps share one table
        uint32_t want = query_cap;
        if (s && want < 2 * s->cap) want = 2 * s->cap < SOGRAND_QUERY_CAP_MAX ? 2 * s->cap : SOGRAND_QUERY_CAP_MAX;
        if (want < 4096) want = 4096 < SOGRAND_QUERY_CAP_MAX ? 4096 : want;
        Schedule *ns = nullptr;
        int rc = build_schedule(code, dev, want, &ns);
        if (rc != SOGRAND_OK && want > query_cap) rc = build_schedule(code, dev, query_cap, &ns);
        if (rc != SOGRAND_OK) return rc;
        if (s) code->retired.push_back(s);
        s = ns;
    }
    dc->hcol = hc;
    for (int c = 0; c < 2; c++) {
        int cl = code->even ? c : 0;
        dc->pat[c] = s->pat[cl];
        dc->wmax[c] = s->wmax[cl];
        dc->len[c] = s->len[cl];
    }
    dc->n = code->n;
    dc->even = code->even;
    dc->phi = code->phi;
    return SOGRAND_OK;
}

}  // namespace sg

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
extern "C" {

const char *sogrand_last_error(void) { return sg::g_last_error.c_str(); }

int sogrand_version(void) { return 100; }

void sogrand_params_default(sogrand_params_t *p) {
    if (!p) return;
    p->list_max = 4;
    p->query_cap = 1000;
    p->alpha = 0.5;
    p->max_iter = 4;
    p->early_stop = 1;
    p->precision = SOGRAND_F64;
    p->list_bler_stop = 0.0;
}

int sogrand_code_create(int n, int k, const uint32_t *h_cols, sogrand_code_t **out) {
    if (!out || !h_cols) return sg::fail(SOGRAND_EINVAL, "NULL argument");
    *out = nullptr;
    if (n < 2 || n > SOGRAND_NMAX) return sg::fail(SOGRAND_EINVAL, "n = %d outside 2..128", n);
    if (k < 1 || n - k < 1 || n - k > 32) return sg::fail(SOGRAND_EINVAL, "need 1 <= n-k <= 32 and k >= 1");
    for (int j = 0; j < n; j++)
        if (n - k < 32 && (h_cols[j] >> (n - k)) != 0)
            return sg::fail(SOGRAND_EINVAL, "h_cols[%d] has bits above row n-k-1", j);
    return sg::make_code(n, k, h_cols, out);
}

int sogrand_code_create_ebch(int n, int k, sogrand_code_t **out) {
    if (!out) return sg::fail(SOGRAND_EINVAL, "NULL argument");
    *out = nullptr;
    uint32_t h[SOGRAND_NMAX];
    int rows = sg::ebch_columns(n, k, h);
    if (rows < 0) return rows;
    if (rows != n - k) SG_TRY(sg::reduce_rows(n, rows, h, n - k));
    return sg::make_code(n, k, h, out);
}

int sogrand_code_info(const sogrand_code_t *code, int *n, int *k, int *is_even, uint32_t *h_cols) {
    if (!code) return sg::fail(SOGRAND_EINVAL, "code is NULL");
    if (n) *n = code->n;
    if (k) *k = code->k;
    if (is_even) *is_even = code->even;
    if (h_cols) std::memcpy(h_cols, code->hcol, sizeof(uint32_t) * code->n);
    return SOGRAND_OK;
}

void sogrand_code_destroy(sogrand_code_t *code) {
    if (!code) return;
    for (auto &kv : code->d_hcol)
        if (kv.second) (void)hipFree(kv.second);
    for (auto &kv : code->sched) sg::free_schedule(kv.second);
    for (auto *s : code->retired) sg::free_schedule(s);
    delete code;
}

}  // extern "C"
