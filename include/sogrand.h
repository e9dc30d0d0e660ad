/*
 * libsogrand -- soft-output GRAND (SOGRAND) decoding of product codes on AMD
 * Instinct MI355X (gfx950).
 *
 * The method is that of Yuan, Medard, Galligan and Duffy, "Soft-output (SO)
 * GRAND and iterative decoding to outperform LDPCs" (arXiv 2310.10737):
 *   - GRAND list decoding: noise-effect patterns are queried in order and a
 *     pattern is a hit when the corrected word passes H c = 0 (section
 *     "Background on GRAND"); the list ends after L hits or a query cap;
 *   - query order: basic ORBGRAND (bits ranked by |LLR|; patterns by
 *     logistic weight = sum of ranks, then Hamming weight, then the rank
 *     tuple in lexicographic order), with the even-code parity skip;
 *   - block soft output: Corollary 1 (eqs. app_approx_correct and
 *     app_approxlist), applied within the parity class for even codes;
 *   - bitwise soft output: eq. (LLRi); L_E = L_APP - L_A - L_Ch (section
 *     "Bitwise SO accuracy", SISO decoder);
 *   - product codes: block turbo decoding with L_A = alpha L_E between row and
 *     column passes and a stop when every row and column of the hard decision
 *     is a codeword (section "Iterative decoding").
 *
 * Conventions used by every call:
 *   - An LLR is log p(bit = 0) / p(bit = 1): positive means bit 0.  A zero LLR
 *     decides bit 0.  BPSK maps bit 0 to +1.
 *   - All functions return 0 (SOGRAND_OK) or a negative SOGRAND_E* code and
 *     never throw; sogrand_last_error() gives a message for the calling thread.
 *   - Buffers named "device" are device memory owned by the caller (for
 *     example torch tensors' data_ptr()); the library never frees them and
 *     never keeps a pointer to them after the call's stream work completes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Decode calls are asynchronous on that stream: they enqueue kernels and
 *     stream-ordered allocations and return without synchronising.  Calls on
 *     different streams may run concurrently; a code handle may be shared.
 *   - Sizes: 2 <= n <= 128, 1 <= n-k <= 32, 1 <= list_max <= 16,
 *     1 <= query_cap <= 2^24.
 */
#ifndef SOGRAND_H
#define SOGRAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SOGRAND_OK 0
#define SOGRAND_EINVAL (-1)    /* bad argument: size, range or NULL pointer      */
#define SOGRAND_ENOMEM (-2)    /* host or device allocation failed               */
#define SOGRAND_EDEVICE (-3)   /* a HIP runtime call or kernel launch failed     */
#define SOGRAND_EAGAIN (-4)    /* serving: admission refused, retry later        */
#define SOGRAND_ENOTFOUND (-5) /* serving: unknown request / nothing completed   */
#define SOGRAND_ETIMEDOUT (-6) /* serving: poll deadline passed                  */

#define SOGRAND_NMAX 128
#define SOGRAND_LIST_MAX 16
#define SOGRAND_QUERY_CAP_MAX (1u << 24)

/* Storage precision of the LLR buffers of a call.  The decoder computes in
   binary64 in both cases; SOGRAND_F32 only reads and writes binary32. */
#define SOGRAND_F64 0
#define SOGRAND_F32 1

/* Message for the last failed call on this thread (never NULL). */
const char *sogrand_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int sogrand_version(void);

/* ------------------------------------------------------------------------ */
/* Codes                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct sogrand_code sogrand_code_t; /* opaque, immutable, library-owned */

/* A binary linear [n, k] code given by its parity-check matrix: h_cols is a
   HOST array of n entries, bit r of h_cols[j] is H[r][j], r < n-k; H must have
   full rank n-k.  Whether the code is even (every codeword of even weight, so
   that only one pattern parity is queried) is derived from H.  The library
   copies h_cols; *out is released with sogrand_code_destroy.
   Errors: EINVAL (sizes, rank), ENOMEM. */
int sogrand_code_create(int n, int k, const uint32_t *h_cols, sogrand_code_t **out);

/* Extended BCH codes of length 2^m: [8,4], [16,11], [32,26], [64,57],
   [128,120] (extended Hamming) and [16,7] (t = 2), built from the primitive
   polynomials x^3+x+1, x^4+x+1, x^5+x^2+1, x^6+x+1, x^7+x^3+1.  Any basis of
   the dual code gives the same decoding.  Errors: EINVAL for other (n, k). */
int sogrand_code_create_ebch(int n, int k, sogrand_code_t **out);

/* n, k, evenness and the n parity-check columns (h_cols may be NULL). */
int sogrand_code_info(const sogrand_code_t *code, int *n, int *k, int *is_even, uint32_t *h_cols);

void sogrand_code_destroy(sogrand_code_t *code);

/* ------------------------------------------------------------------------ */
/* Parameters                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int list_max;       /* L: stop after this many codewords, 1..16                */
    uint32_t query_cap; /* stop after this many tested patterns, 1..2^24          */
    double alpha;       /* product codes: L_A = alpha * L_E, > 0 (paper: 0.5)     */
    int max_iter;       /* product codes: full row+column iterations, 1..1000     */
    int early_stop;     /* product codes: stop once the hard decision is valid    */
    int precision;      /* SOGRAND_F64 or SOGRAND_F32 LLR storage                 */
    double list_bler_stop; /* 0 (off) or a threshold in (0, 1]: a word's search also
                           ends after a codeword whose list so far has a predicted
                           list-BLER (Corollary 1, with the mass tested up to that
                           query) below it; the paper's figures use 1e-4..1e-6 */
} sogrand_params_t;

/* Fills the paper's settings: L = 4, cap 1000, alpha 0.5, 4 iterations,
   early stop on, binary64 storage, no list-BLER stop. */
void sogrand_params_default(sogrand_params_t *p);

/* ------------------------------------------------------------------------ */
/* Component SISO decoding (section "Bitwise SO accuracy", Fig. SISO)       */
/* ------------------------------------------------------------------------ */
/* Decodes nwords independent words.  llr_in is the SISO input
   lambda = L_Ch + L_A, DEVICE, row-major [nwords][n], binary64 or binary32 per
   params->precision.  Outputs, all DEVICE and each optional (NULL = not written):
     llr_app  [nwords][n]            L_APP by eq. (LLRi), clamped to +-1000
     llr_ext  [nwords][n]            L_E = L_APP - lambda
     hard     [nwords][n]  uint8     1 iff L_APP < 0
     n_queries[nwords]     uint32    patterns tested (the query count)
     n_found  [nwords]     uint8     codewords in the list (<= list_max)
     found_q  [nwords][list_max]     query number of each found codeword
     p_found  [nwords][list_max]     APP of each found codeword (Corollary 1)
     p_notfound [nwords]   double    probability the codeword is not in the list
     found_z  [nwords][list_max][n]  uint8 error pattern of each found codeword
   Entries of found_q / p_found / found_z past n_found are written as zero.
   Errors: EINVAL (params, sizes, llr_in NULL), ENOMEM, EDEVICE. */
int sogrand_decode_component(const sogrand_code_t *code, const sogrand_params_t *params,
                             size_t nwords, const void *llr_in, void *llr_app, void *llr_ext,
                             uint8_t *hard, uint32_t *n_queries, uint8_t *n_found,
                             uint32_t *found_q, double *p_found, double *p_notfound,
                             uint8_t *found_z, void *stream);

/* ------------------------------------------------------------------------ */
/* Product codes: block turbo decoding (section "Iterative decoding")       */
/* ------------------------------------------------------------------------ */
/* Decodes nframes frames of an (n^2, k^2) product code whose rows and columns
   are words of `code`.  llr_ch: DEVICE [nframes][n][n] channel LLRs (row-major,
   precision per params).  Half-iteration h = 1, 2, ... decodes every row (h
   odd) or column (h even) of L_Ch + L_A; after each, the hard decision of
   L_APP is tested (every row and column a codeword) and, unless the frame
   stops, L_A = alpha * L_E.  Outputs (DEVICE):
     hard      [nframes][n][n] uint8  final hard decision (required)
     llr_app   [nframes][n][n]        final L_APP (optional, precision per params)
     success   [nframes] uint8        1 iff the final hard decision is valid (required)
     half_iters[nframes] uint16       half-iterations run (optional)
     sum_queries     [nframes] uint64 patterns tested over all words (optional)
     sum_max_queries [nframes] uint64 sum over half-iterations of the largest
                                      per-word query count (optional)
   The library allocates its work buffers stream-ordered on `stream`.
   Errors: EINVAL, ENOMEM, EDEVICE. */
int sogrand_decode_product(const sogrand_code_t *code, const sogrand_params_t *params,
                           size_t nframes, const void *llr_ch, uint8_t *hard, void *llr_app,
                           uint8_t *success, uint16_t *half_iters, uint64_t *sum_queries,
                           uint64_t *sum_max_queries, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   decoding as sogrand_decode_product, with identical results, but the work
   buffer is a static device array of SOGRAND_NOALLOC_WORK_MAX bytes that the
   library holds on each device it has run this call on, until the process ends.
   The call allocates nothing (no hipMalloc, hipFree or stream-ordered
   allocation) and leaves the measurement hooks out.
   Limits and preconditions:
     - the work buffer of nframes frames of length n, about
       nframes * (3 n^2 b + 16 n + 32) bytes with b = 8 (F64) or 4 (F32) LLR
       storage, must fit in SOGRAND_NOALLOC_WORK_MAX bytes (else EINVAL; for
       example 1300 [64,57]^2 frames in binary32, 170 [128,120]^2 frames in
       binary64);
     - the code's device tables for this device and a query cap at least
       params->query_cap must exist, built by any earlier allocating decode call
       (component, product, QC-GLDPC, batched or serving) with this code on this
       device (else EINVAL);
     - every call on one device shares that device's array, and nothing is kept
       from one call to the next: calls whose work overlaps on one device (other
       streams, or other threads) race and give wrong results; serialise them.
   Arguments, outputs and the other errors as for sogrand_decode_product. */
#define SOGRAND_NOALLOC_WORK_MAX (64u << 20)
int sogrand_decode_product_noalloc(const sogrand_code_t *code, const sogrand_params_t *params,
                                   size_t nframes, const void *llr_ch, uint8_t *hard, void *llr_app,
                                   uint8_t *success, uint16_t *half_iters, uint64_t *sum_queries,
                                   uint64_t *sum_max_queries, void *stream);

/* ------------------------------------------------------------------------ */
/* QC-GLDPC codes (section "Performance evaluation", GLDPC decoding)        */
/* ------------------------------------------------------------------------ */
/* Decodes nframes frames of the (n^2, n^2 - 2n(n-k)) quasi-cyclic GLDPC code
   whose adjacency matrix has the block rows [I(0) ... I(0)] and
   [I(0) I(1) ... I(n-1)], I(i) the n x n identity rotated right by i positions,
   with `code` at every check node.  Variable node j*n + c is column c of block
   j; check node r of the first block row takes its bit j from variable node
   j*n + r, check node r of the second from j*n + (r + j) mod n.  llr_ch: DEVICE
   [nframes][n*n] channel LLRs by variable node (precision per params).
   Decoding is the block turbo loop of sogrand_decode_product with the two
   block rows in place of rows and columns: half-iteration h decodes every
   check node of the first (h odd) or second (h even) block row on L_Ch + L_A,
   each variable node taking L_A = alpha * L_E from its check node in the other
   block row; after each half the hard decision of L_APP is tested (every check
   node of both block rows a codeword).  The paper's GLDPC runs use alpha = 0.6,
   max_iter = 20 and list_bler_stop = 1e-5.  Outputs, by variable node, and
   errors as for sogrand_decode_product. */
int sogrand_decode_gldpc(const sogrand_code_t *code, const sogrand_params_t *params,
                         size_t nframes, const void *llr_ch, uint8_t *hard, void *llr_app,
                         uint8_t *success, uint16_t *half_iters, uint64_t *sum_queries,
                         uint64_t *sum_max_queries, void *stream);

/* ------------------------------------------------------------------------ */
/* Plans: a decode's launches captured once in a HIP graph                  */
/* ------------------------------------------------------------------------ */
/* The block turbo decoding of sogrand_decode_product (section "Iterative
   decoding"), or of sogrand_decode_gldpc when gldpc is nonzero, over nframes
   frames whose buffers are fixed when the plan is made.  create records the
   decode's kernel launches (the initialisation, then a pass and a validity check
   per half-iteration: 4 max_iter + 1 launches) into a HIP graph once, and
   allocates the plan's own work buffer (the only allocation); it builds the
   code's tables if needed and returns when done.  Arguments are those of
   sogrand_decode_product (DEVICE buffers, same shapes, layouts and optional
   outputs); they must stay valid while the plan exists.  launch enqueues one
   replay of the graph on `stream`, on the device current at create: the frames
   that llr_ch holds when it runs are decoded into the plan's outputs exactly as
   sogrand_decode_product would decode them.  It saves the per-launch cost of the
   separate launches, which counts when frames are few.  Launches of one plan
   share its work buffer and outputs, so they must not overlap (use one stream,
   or order them).  destroy frees the plan after waiting for the device; it
   accepts NULL.  Errors: EINVAL (also for nframes 0), ENOMEM, EDEVICE. */
typedef struct sogrand_plan sogrand_plan_t;
int sogrand_plan_create(const sogrand_code_t *code, const sogrand_params_t *params, size_t nframes, int gldpc,
                        const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success, uint16_t *half_iters,
                        uint64_t *sum_queries, uint64_t *sum_max_queries, sogrand_plan_t **out);
int sogrand_plan_launch(sogrand_plan_t *plan, void *stream);
void sogrand_plan_destroy(sogrand_plan_t *plan);

/* ------------------------------------------------------------------------ */
/* Batched decoding: mixed codes, one persistent launch                     */
/* ------------------------------------------------------------------------ */
/* Launch shape of the persistent kernel.  Each workgroup (waves_per_group
   waves) keeps frames_per_group frames in flight and its waves take
   steal_chunk rows or columns at a time from whichever of them has lines left
   in its current half-iteration; at most groups_per_cu workgroups run per compute
   unit, and no more than fit on it at once.  Every frame is decoded exactly as by
   sogrand_decode_product, so results do not depend on the shape. */
typedef struct {
    int waves_per_group;   /* 4, 8 or 16 */
    int frames_per_group;  /* 1..8 */
    int steal_chunk;       /* 1..128 */
    int groups_per_cu;     /* 1..64 */
} sogrand_sched_t;

/* A measured default (8 waves, 2 frames, 4 lines, as many groups per CU as fit). */
void sogrand_sched_default(sogrand_sched_t *s);

/* Block turbo decoding (section "Iterative decoding") of nframes frames whose
   codes may differ.  codes: HOST array of ncodes (1..8) code handles.
   frame_code[f] (DEVICE, uint8) indexes codes; frame_offset[f] (DEVICE) is the
   element offset of frame f's n x n row-major block in llr_ch (DEVICE, llr_len
   elements, precision per params), in hard (DEVICE, llr_len bytes: the final hard
   decision, written once when the frame finishes) and in llr_app (DEVICE, llr_len
   elements in the params precision, optional: the final L_APP).  Per-frame outputs
   (DEVICE) as in sogrand_decode_product; success is required, the others may be
   NULL.  status (DEVICE, optional) receives 0, or bit 0 if a wave gave up waiting
   (not expected) and bit 1 if a frame descriptor was out of range (that frame is
   skipped with success 0 and half_iters 0, and its hard and llr_app are not
   written).  Frames are taken longest code first and, among the frames of the
   shortest code, those with the smallest mean |L_Ch| over their first 1024
   elements first (a sort on the device), so that the end of the launch is left
   to short, easy frames; the order changes no result.  sched NULL = the shape recorded for this kind of batch by
   sogrand_sched_tune or sogrand_sched_table_load, else the default adjusted to the
   batch's size: up to one frame per compute unit, 16-wave workgroups of one frame
   taking 2 lines per steal; up to eight frames per compute unit, one frame per
   workgroup.  Errors:
   EINVAL, ENOMEM, EDEVICE. */
int sogrand_decode_batched(const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                           size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset,
                           uint64_t llr_len, const void *llr_ch, uint8_t *hard, void *llr_app, uint8_t *success,
                           uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                           uint32_t *status, const sogrand_sched_t *sched, void *stream);

/* The same persistent decoding of QC-GLDPC frames (performance-evaluation
   section; frames laid out by variable node as for sogrand_decode_gldpc): frame
   f's n x n block at frame_offset[f] holds variable node j*n + c at element
   [j][c], and its code's n words of the first block row and n of the second
   alternate as the rows and columns of a product frame do.  Every frame is
   decoded exactly as by sogrand_decode_gldpc.  Arguments, outputs and errors as
   for sogrand_decode_batched. */
int sogrand_decode_batched_gldpc(const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                                 size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset,
                                 uint64_t llr_len, const void *llr_ch, uint8_t *hard, void *llr_app,
                                 uint8_t *success,
                                 uint16_t *half_iters, uint64_t *sum_queries, uint64_t *sum_max_queries,
                                 uint32_t *status, const sogrand_sched_t *sched, void *stream);

/* Launch-shape tuner for the persistent kernel.  Decodes the sample described by
   the arguments (as for sogrand_decode_batched, or sogrand_decode_batched_gldpc
   when gldpc is nonzero; the outputs go to buffers of the tuner's own) once per
   candidate shape and times each with HIP events on `stream`.  The candidates
   come from a coordinate search that starts at the default and varies
   waves_per_group over {4, 8, 16}, frames_per_group over {1, 2, 3, 4} and
   steal_chunk over {1, 2, 4, 8} in turn, keeping a change when it is faster;
   groups_per_cu stays at the default (as many as fit).  The fastest shape goes
   to *best, its time in milliseconds to *best_ms (optional), and the library's
   table of tuned shapes, under the batch's kind: topology, precision, whether
   the list-BLER stop is on, and the (n, k) of its codes.  A later batched call
   with sched NULL on a batch of that kind uses it.  The sample should look like
   the batches the shape will serve, in size too: the end of a launch, where the
   last frames drain, weighs more in a small sample.  Blocks until done; results
   of a decode never depend on the shape.  Errors: EINVAL (also for an empty sample),
   ENOMEM, EDEVICE. */
int sogrand_sched_tune(int gldpc, const sogrand_code_t *const *codes, int ncodes, const sogrand_params_t *params,
                       size_t nframes, const uint8_t *frame_code, const uint64_t *frame_offset, uint64_t llr_len,
                       const void *llr_ch, sogrand_sched_t *best, float *best_ms, void *stream);

/* The table of tuned shapes as a text file: one line per batch kind, the kind's
   name, '|', then waves_per_group frames_per_group steal_chunk groups_per_cu.
   save writes every entry (EINVAL if the file cannot be written); load adds the
   file's entries, replacing those of the same kind, and returns how many it read
   (EINVAL for an unreadable file or a malformed or out-of-range line, in which
   case nothing is added); clear empties the table. */
int sogrand_sched_table_save(const char *path);
int sogrand_sched_table_load(const char *path);
void sogrand_sched_table_clear(void);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of product-frame decode requests            */
/* ------------------------------------------------------------------------ */
/* A server owns a pool of frame slots in device memory (hbm_budget_bytes) and
   four lanes: host threads with their own HIP streams that each advance their
   frames by one half-iteration per step (section "Iterative decoding").  In a
   step the row or column pass of all the lane's frames, whatever their codes,
   runs in one launch, followed by the validity check launch.  Frames that
   finish leave, and requests submitted meanwhile join the next lane to start a
   step, so new work overlaps with frames already in flight.  Each frame is
   decoded exactly as sogrand_decode_product decodes it alone.

   A slot holds the frame's channel LLRs, a-priori LLRs, hard decision and
   line syndromes; its size is set by the code length rounded up to 32, 64 or
   128.  A host copy of equal size (pinned memory) carries the LLRs in and the
   hard decisions out.  The server decodes on the device current at creation.

   The lanes' steps run concurrently only if their streams sit on different
   hardware queues.  HIP gives a process four by default (GPU_MAX_HW_QUEUES), and
   streams created once others hold queues share them: create the server before
   the process's other streams (including the default stream's first use), or
   raise GPU_MAX_HW_QUEUES.  On an MI355X a server created after other GPU work
   with four queues ran its steps at 0.20 ms on average instead of 0.15. */
typedef struct sogrand_server sogrand_server_t;

typedef struct {
    uint64_t request_id;
    uint64_t user_tag;
    int32_t status;          /* 0, or SOGRAND_EDEVICE if the device failed       */
    uint8_t success;         /* hard decision is a product codeword              */
    uint16_t half_iters;     /* half-iterations run                              */
    uint16_t n;              /* code length: the result's hard decision is n*n bytes */
    uint64_t queries;        /* patterns tested over all words and half-iterations */
    uint64_t hard_offset;    /* byte offset of the hard decision in hard_out_host */
    uint64_t t_submit_ns;    /* sogrand_clock_ns() at submission                 */
    uint64_t t_admit_ns;     /* ... when the frame entered its first step        */
    uint64_t t_done_ns;      /* ... when its last step completed                 */
} sogrand_result_t;

/* CLOCK_MONOTONIC in nanoseconds: the clock of the result timestamps. */
uint64_t sogrand_clock_ns(void);

/* Server flag: keep every frame's L_APP of its last half-iteration and return it
   with the result (sogrand_serve_poll's llr_app_out_host).  A slot then also holds
   n*n LLRs of the server's precision. */
#define SOGRAND_SERVE_APP 1u

/* params as for sogrand_decode_product (precision sets the LLR storage of the
   slots and of llr_ch_host).  hbm_budget_bytes: device memory for slots, at
   least 1 MiB; the same amount of pinned host memory is allocated.  flags: 0 or
   SOGRAND_SERVE_APP.  Errors: EINVAL, ENOMEM, EDEVICE. */
int sogrand_serve_create(const sogrand_params_t *params, size_t hbm_budget_bytes, unsigned flags,
                         sogrand_server_t **out);

/* Admits one frame: llr_ch_host is HOST memory, n*n LLRs row-major in the
   server's precision, copied before the call returns (the caller keeps it).
   A server accepts up to 16 distinct codes.  Returns SOGRAND_EAGAIN when no
   slot is free (poll for results, then retry), EINVAL for bad arguments or a
   seventeenth code, EDEVICE after a device failure. */
int sogrand_serve_submit(sogrand_server_t *server, const sogrand_code_t *code, const void *llr_ch_host,
                         uint64_t user_tag, uint64_t *request_id);

/* Takes up to max_results finished requests, oldest first, waiting up to
   timeout_ns (0: do not wait; < 0: until one finishes).  If hard_out_host is
   not NULL it receives each result's n*n hard decisions at hard_offset, packed
   back to back (at most max_results * 16384 bytes).  If llr_app_out_host is not
   NULL and the server was created with SOGRAND_SERVE_APP, it receives each
   result's n*n final L_APP (row-major, the server's precision) at element offset
   hard_offset (at most max_results * 16384 elements); HOST memory, caller-owned.
   Returns SOGRAND_OK with *n_results >= 1, SOGRAND_ETIMEDOUT if none finished in
   time, SOGRAND_ENOTFOUND if nothing is in flight and nothing is waiting to be
   taken. */
int sogrand_serve_poll(sogrand_server_t *server, sogrand_result_t *results, size_t max_results,
                       size_t *n_results, uint8_t *hard_out_host, void *llr_app_out_host, int64_t timeout_ns);

/* Open-loop load generator for measurement: submits request i (code
   codes[req_code[i]], LLRs at element offset req_offset[i] of llr_host, HOST
   memory of llr_len elements) at time t0_ns + arrival_ns[i] on sogrand_clock_ns(), with user_tag i,
   busy-waiting until it is due; a refused request (no free slot) is retried
   until admitted, so its wait counts in its latency.  Blocks until every
   request is submitted; results are taken with sogrand_serve_poll from another
   thread meanwhile.  *retries (optional) counts refused attempts.
   Errors: EINVAL, EDEVICE. */
int sogrand_serve_replay(sogrand_server_t *server, const sogrand_code_t *const *codes, int ncodes, size_t nreq,
                         const uint8_t *req_code, const uint64_t *req_offset, const void *llr_host,
                         uint64_t llr_len, const uint64_t *arrival_ns, uint64_t t0_ns, uint64_t *retries);

/* Counters since creation. */
typedef struct {
    uint64_t steps;        /* steps run                                          */
    uint64_t frames;       /* frames finished                                    */
    uint64_t max_active;   /* most frames advanced by one step                   */
    double step_ms;        /* summed step time, first launch to completion       */
    double max_step_ms;    /* longest step                                       */
    double host_ms;        /* summed host time outside steps while work was admitted
                              (admission, result hand-off)                       */
} sogrand_serve_stats_t;

int sogrand_serve_stats(sogrand_server_t *server, sogrand_serve_stats_t *stats);

/* Finishes every admitted request, then releases the server; results not
   taken are discarded. */
int sogrand_serve_destroy(sogrand_server_t *server);

/* ------------------------------------------------------------------------ */
/* Measurement                                                              */
/* ------------------------------------------------------------------------ */
/* Per-kernel-family totals collected between sogrand_profile_begin and
   sogrand_profile_end (process-wide, all devices and streams). */
typedef struct {
    char kernel[48];     /* family: "component", "product_pass", "product_check", ... */
    uint64_t launches;   /* kernel launches recorded                                  */
    double total_ms;     /* sum of HIP-event times around those launches              */
    uint64_t words;      /* component words decoded (count_work only)                 */
    uint64_t queries;    /* patterns tested (count_work only)                         */
    uint64_t ranks;      /* sum of the Hamming weights of the tested patterns (count_work only) */
    uint64_t exact_rank; /* words whose ranks needed the exact tie-resolving pass (count_work only) */
    uint64_t phase_cycles[8]; /* count_work in a build with SG_PHASE_CLOCKS defined, else 0: wave clock
                                 cycles spent per decode phase, summed over words: hard decision,
                                 syndrome and rho; ranking; class masses; query loop; soft output; the
                                 rest of the word's work in the kernel (inputs, outputs); in the
                                 persistent kernel, cycles spent finding work (claims, waiting) and on
                                 half-iteration hand-overs (validity check, retire, refill) */
} sogrand_kernel_stat_t;

/* Starts recording: every decode kernel launched afterwards is bracketed by a
   pair of HIP events on its stream.  With count_work != 0 the kernels also add
   the words, queries and pattern weights they process to device counters
   (this adds atomics; use a separate run for timing).  Errors: EDEVICE. */
int sogrand_profile_begin(int count_work);

/* Stops recording, waits for the recorded events and returns up to max_stats
   families in stats (*n_stats set).  Errors: EINVAL, EDEVICE. */
int sogrand_profile_end(sogrand_kernel_stat_t *stats, int max_stats, int *n_stats);

/* Measures the device's VALU issue rate for one instruction kind: a kernel of
   eight independent chains per lane (64 VALU instructions per loop trip, eight
   waves on every SIMD) runs four times on `stream` (NULL: the null stream) after
   a warm-up.  kind 0: 32-bit XOR and ADD (VOP2 forms), the measured counterpart
   of the ALU roofline's derived peak; 1: binary64 FMA; 2: 32-bit bit-field
   extract and shift-add (VOP3 forms).  Returns lane-operations (one per lane per instruction) per second in
   *lane_ops_per_s and the mean launch time in *ms (nullable).  Blocks until
   done.  Errors: EINVAL, ENOMEM, EDEVICE. */
int sogrand_measure_valu_rate(int kind, double *lane_ops_per_s, double *ms, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SOGRAND_H */
