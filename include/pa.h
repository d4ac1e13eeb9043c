/*
 * libpa: the G_{c,d} privacy-amplification hash on an MI355X (gfx950) GPU.
 *
 * The hash is the modular-arithmetic universal_2 family of Section 2.3,
 * eq. (6) and the g_{c,d} definition after it:
 *
 *     G_{c,d} = { g_{c,d} : c, d in Z_{2^n}, c odd },
 *     g_{c,d}(x) = floor( ((c x + d) mod 2^n) / 2^(n - m) ),
 *
 * evaluated in the order of the scheme of Section 3.2: multiply-add (3.2.2),
 * reduction mod 2^n (3.2.3), export (3.2.4) and selection of the most
 * significant r = m bits (3.2.5).  x is the n-bit corrected key, the output is
 * the m-bit final key.  The large multiply is an exact NTT convolution (the
 * approach of Alg. 1) of 64-bit digits over five 31-bit primes or 96-bit
 * digits over seven, whichever needs less transform work for the block, done
 * by HIP kernels.
 *
 * Bit layout (all arrays): little-endian 64-bit words, word 0 least
 * significant; bit i of a value is bit (i % 64) of word i / 64.  Inputs have
 * ceil(n/64) words and bits >= n of their top word are ignored.  Outputs have
 * ceil(m/64) words and bits >= m of the top word are written as 0.  Output bit
 * j is bit (n - m + j) of V = (c x + d) mod 2^n; leading zeros of V count.
 *
 * Seeds (the paper chooses g at random and publicly, Section 2.2): word i of
 * the stream of seed s is the i-th output of SplitMix64(s) (Steele, Lea and
 * Flood, OOPSLA 2014).  c is the stream of seed_a masked to n bits with bit 0
 * set; d is the stream of seed_b masked to n bits.  This generator is not
 * cryptographic: a deployment passes true random c and d through pa_hash_ex.
 *
 * Errors: every call returns PA_OK or a PA_E* code; no exception crosses the
 * ABI.  On error the output is unspecified and the context stays usable;
 * pa_last_error() gives a text for the last failure on that context.
 *
 * Ownership and threads: the caller owns every key, operand and output buffer.
 * A context owns its device workspace, tables and stream and frees them in
 * pa_destroy().  A context is not thread-safe; several contexts may coexist.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pa_status {
    PA_OK = 0,
    PA_EINVAL = 1,   /* null pointer, n == 0, m == 0, m > n, n > PA_MAX_N, even c */
    PA_ENOMEM = 2,   /* host or device allocation failed */
    PA_EDEVICE = 3,  /* a HIP runtime call failed (see pa_last_error) */
    PA_ENODEV = 4,   /* no usable gfx950 device with that index */
    PA_EIO = 5,      /* the tuning cache file could not be read or written */
};

/* Largest block: 2^23 64-bit digits (transform length 2^24; the coefficient
 * bound 2^23 2^128 stays below the five primes' product, 2^153.4). */
#define PA_MAX_N ((uint64_t)1 << 29)

typedef struct pa_ctx pa_ctx;

/*
 * Context options (pa_init; NULL gives the defaults: no budget, no cache).
 *   hbm_budget: the device bytes the context may hold for itself: its twiddle
 *     tables (0.8 MB), the block workspace (pa_workspace_bytes of the largest
 *     block so far), the host-transfer staging buffers, the Toeplitz t buffer
 *     and pa_tune's two temporary buffers.  A call that would grow them past
 *     it fails with PA_ENOMEM before allocating and leaves the context usable.
 *     0: no limit.  Batches (pa_batch_bytes), cached multipliers and servers
 *     are objects of their own, outside it.
 *   tune_cache: path of a text file of tuned geometries.  pa_init applies the
 *     file's entries for this GPU architecture (as pa_plan_set would; a
 *     missing file is an empty cache, an unreadable one PA_EIO), and every
 *     pa_tune appends its result as one line
 *       pa_tune <arch> <W> <f> <k> <tile_log> <strided_tile_log> <rows3_log> <ms>
 *     (digit words W, transform length f 2^k).  Later lines override earlier
 *     ones; lines of another architecture or format, or whose geometry is not
 *     valid for the length, are ignored.  NULL: no file.  The matching of the
 *     multiplication method to the operand size that the paper leaves to GMP
 *     (Sections 2.3 and 3.2.2) is this measurement, kept across processes.
 */
typedef struct pa_opts {
    uint64_t hbm_budget;
    const char *tune_cache;
} pa_opts;

/* Create a context on HIP device `device` (its own stream and tables). */
int pa_init(pa_ctx **ctx, int device, const pa_opts *opts);

/* Device bytes the context holds now (what hbm_budget bounds). */
uint64_t pa_ctx_bytes(const pa_ctx *ctx);

/* Wait for the device (work queued on any stream, including callers' streams
 * through the _async calls), then release the context and everything it owns.
 * NULL is allowed. */
void pa_destroy(pa_ctx *ctx);

/* Static text for a status code. */
const char *pa_strerror(int status);

/* Text describing the last failure on ctx (empty if none). */
const char *pa_last_error(const pa_ctx *ctx);

/*
 * Synchronous, host memory in and out.
 *   key:  ceil(n/64) words (host), the n-bit corrected key x
 *   out:  ceil(m/64) words (host), written with the m-bit final key
 * c and d are expanded from seed_a and seed_b on the device.
 */
int pa_hash(pa_ctx *ctx, const uint64_t *key, uint64_t seed_a, uint64_t seed_b,
            uint64_t n, uint64_t m, uint64_t *out);

/*
 * Synchronous with explicit operands (host memory): c and d are ceil(n/64)
 * words each.  c must be odd (eq. (6)); an even c returns PA_EINVAL.
 */
int pa_hash_ex(pa_ctx *ctx, const uint64_t *key, const uint64_t *c, const uint64_t *d,
               uint64_t n, uint64_t m, uint64_t *out);

/*
 * Asynchronous, device memory: the same g_{c,d} (Section 2.3, eq. (6) and the
 * definition after it; the steps of Section 3.2) with c and d expanded from
 * the seeds.  d_key (ceil(n/64) words) and d_out (ceil(m/64) words) are
 * device pointers; the work is queued on `stream` (a hipStream_t,
 * NULL for the null stream) and the call returns without waiting.  The
 * context's workspace is reused by every call, so calls on one context must
 * be ordered (one stream, or the caller synchronises between streams).  The
 * workspace grows, with a device synchronisation, when n exceeds every
 * earlier call; pa_reserve() avoids that inside a timed or captured region.
 */
int pa_hash_async(pa_ctx *ctx, const uint64_t *d_key, uint64_t seed_a, uint64_t seed_b,
                  uint64_t n, uint64_t m, uint64_t *d_out, void *stream);

/*
 * Allocation-free variant of pa_hash_async, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, result and stream ordering as
 * pa_hash_async, and the same kernels; the block's two spectra and carry state
 * live in a fixed scratch area of PA_NOALLOC_MAX_BYTES on each GPU instead of
 * the context's workspace.  That area is set aside when the library's code is
 * loaded on a GPU and held until the process ends; pa_init takes its address.
 * The call allocates and frees nothing and never synchronises.
 *   Limit: a block needs its spectra and carry state (pa_workspace_bytes(n),
 *   plus at most 768 bytes of alignment) to fit; every n up to 3 * 2^25 =
 *   100 663 296 bits does (the paper's largest block, 10^8 bits, included).
 *   Larger n returns PA_EINVAL with the sizes in pa_last_error.
 *   Sharing: every call on one GPU, from any context or thread, uses that
 *   GPU's one scratch area, which keeps the last call's contents (nothing in
 *   it needs to start at zero).  Calls that overlap on one GPU race and give
 *   wrong results: order them on one stream or synchronise between them.
 */
#define PA_NOALLOC_MAX_BYTES ((uint64_t)120 << 20)
int pa_hash_async_noalloc(pa_ctx *ctx, const uint64_t *d_key, uint64_t seed_a, uint64_t seed_b,
                          uint64_t n, uint64_t m, uint64_t *d_out, void *stream);

/*
 * Per-launch timing of one pa_hash_async call, for measurement.  The same
 * kernels run as in pa_hash_async on `stream`; each launch carries a start and
 * stop event stamped by its own dispatch (hipExtLaunchKernelGGL, so nothing
 * is queued between the kernels), and the call waits for the stream before
 * returning.
 *   kind:  PA_K_* of each launch
 *   ms:    its duration from the events
 *   bytes: the bytes the launch must move at minimum (its algorithmic traffic)
 */
#define PA_PROFILE_MAX 32
enum pa_kernel_kind {
    PA_K_NTT_PASS = 0,    /* one LDS pass of a forward, fused or inverse NTT */
    PA_K_CARRY_LOCAL = 1, /* CRT + addend + column sums -> carry function per chunk */
    PA_K_CARRY_APPLY = 3, /* carry-in from the chunk functions, CRT + addend + resolve + mod 2^n + top-m */
};
typedef struct pa_profile {
    int count;
    int kind[PA_PROFILE_MAX];
    float ms[PA_PROFILE_MAX];
    uint64_t bytes[PA_PROFILE_MAX];
} pa_profile;

int pa_hash_profile(pa_ctx *ctx, const uint64_t *d_key, uint64_t seed_a, uint64_t seed_b,
                    uint64_t n, uint64_t m, uint64_t *d_out, void *stream, pa_profile *prof);

/*
 * Cached multiplier (opt-in).  When the same multiplier c is used for many
 * blocks of one size n, its transform can be computed once and kept on the
 * device; each block then needs two transforms instead of three.  The paper
 * does not say whether g may be reused across blocks (Section 2.2 has it
 * chosen at random and publicly); reuse is the caller's security decision.
 *   pa_mul_create: transform c (expanded from seed_a, or the device words d_c,
 *     which must be odd) for blocks of n bits, queued on `stream`.  With d_c
 *     it first reads c's low word in `stream` order and waits for it.
 *   pa_hash_mul_async: hash the device key d_key (ceil(n/64) words) with that
 *     c and the addend of seed_b; m output bits into d_out.  Same ordering
 *     rules as pa_hash_async (the context's workspace is reused).  ctx may be
 *     any context on the device the multiplier was made on (else PA_EINVAL).
 *   pa_mul_destroy: waits for the device, then frees the spectrum; it may
 *     come before or after pa_destroy of the creating context.
 */
typedef struct pa_mul pa_mul;
int pa_mul_create(pa_ctx *ctx, uint64_t seed_a, const uint64_t *d_c, uint64_t n, void *stream,
                  pa_mul **mul);
int pa_hash_mul_async(pa_ctx *ctx, const pa_mul *mul, const uint64_t *d_key, uint64_t seed_b,
                      uint64_t m, uint64_t *d_out, void *stream);
void pa_mul_destroy(pa_mul *mul);

/*
 * Batches: many blocks of uneven n hashed together.  Blocks are grouped by
 * transform length (and digit layout).  Two ways to run them:
 *   PA_BATCH_GROUPED (the default): every kernel of a group is one launch for
 *     all of the group's blocks; groups run on side streams.
 *   PA_BATCH_PERSISTENT (switched off: creating such a batch returns
 *     PA_EINVAL until the kernel has been validated on a GPU): one
 *     persistent kernel runs everything.
 *     Its workgroups, as many as fit on the device at once, take work items
 *     (one pass tile of one prime of one block, or one carry chunk of one
 *     block) from a device queue in dependency order.  Each item waits until
 *     the items its block needs are done (per-block counters), so different
 *     blocks' passes and carries overlap with no launch boundaries between
 *     them.  The waits are bounded; a run whose wait gave up is reported by
 *     pa_batch_result (never expected; it would leave outputs incomplete).
 * Both compute the same bits as hashing each block alone (the per-block
 * method of Section 2.3, eq. (6), batched).  A group uses the geometry that
 * pa_tune or pa_plan_set chose for its length on the context, if any; else a
 * default for many blocks.  All pointers in a pa_job are device memory.
 *   key:  ceil(n/64) words;  out: ceil(m/64) words
 *   c, d: explicit operands (ceil(n/64) words each) or NULL to expand them
 *         from seed_a / seed_b; an explicit c must be odd (eq. (6))
 *   status: written by pa_batch_create / pa_hash_many: PA_OK, or the reason
 *         the block was left out (its output is then untouched)
 */
typedef struct pa_job {
    const uint64_t *key;
    const uint64_t *c;
    const uint64_t *d;
    uint64_t seed_a, seed_b;
    uint64_t n, m;
    uint64_t *out;
    int status;
} pa_job;

typedef struct pa_batch pa_batch;

/*
 * Validate and plan a batch, allocate its device workspace (one slab for all
 * blocks; see pa_batch_bytes) and upload its job table.  Invalid blocks get
 * their status and are skipped; the call fails only if nothing can run (or on
 * allocation / device errors).  The batch keeps the pointers of `jobs`, not
 * the array itself; the buffers they point to must outlive the batch.  The
 * low word of each explicit c is read here with a synchronous copy, so c must
 * already be written.  Runs and captures need `ctx`; pa_batch_destroy does
 * not, and may follow pa_destroy(ctx).
 */
int pa_batch_create(pa_ctx *ctx, pa_job *jobs, size_t count, pa_batch **batch);

/* Batch options.  NULL gives the defaults (grouped). */
#define PA_BATCH_PERSISTENT 0
#define PA_BATCH_GROUPED 1
typedef struct pa_batch_opts {
    int mode;              /* PA_BATCH_PERSISTENT or PA_BATCH_GROUPED */
    uint32_t wait_us;      /* persistent: microseconds a dependency wait may take before the
                            * run gives up (0: 2 s) */
    int force_abort;       /* persistent, for testing the failure path: every wait for a
                            * dependency gives up at once, and the run reports PA_EDEVICE */
} pa_batch_opts;
int pa_batch_create_ex(pa_ctx *ctx, pa_job *jobs, size_t count, const pa_batch_opts *opts,
                       pa_batch **batch);

/* After the stream of a run has completed: PA_OK, or PA_EDEVICE if the
 * persistent kernel gave up a dependency wait (the outputs are then
 * incomplete).  Needs the batch's context. */
int pa_batch_result(const pa_batch *batch);

/* Queue every kernel of the batch on `stream` (replays the captured graph if
 * pa_batch_capture was called).  Returns without waiting. */
int pa_batch_run(pa_batch *batch, void *stream);

/* Record the batch's launches into a HIP graph on `stream` (NULL: the
 * context's stream) so that later pa_batch_run calls replay it with one
 * launch.  Nothing runs during the capture. */
int pa_batch_capture(pa_batch *batch, void *stream);

/* Device bytes the batch holds (workspace, job table, persistent queue table). */
uint64_t pa_batch_bytes(const pa_batch *batch);

/* Number of blocks that will run, and of kernel launches one run queues
 * (persistent: 2, the counter reset and the queue kernel). */
size_t pa_batch_size(const pa_batch *batch);
size_t pa_batch_launches(const pa_batch *batch);

void pa_batch_destroy(pa_batch *batch);

/* g_{c,d} (Section 2.3, eq. (6) and the definition after it; the steps of
 * Section 3.2) of every block of `jobs`: create (grouped) + run + wait +
 * pa_batch_result + destroy; per-block status in jobs[i].status.  Returns
 * PA_OK if every valid block was hashed (invalid ones only get their status),
 * else the first failure's code. */
int pa_hash_many(pa_ctx *ctx, pa_job *jobs, size_t count, void *stream);

/*
 * Server: continuous hashing of a stream of requests on one GPU.  Requests are
 * admitted in arrival order as soon as one of `slots` slots is free and their
 * device footprint fits in `hbm_budget` bytes (allocated once at creation);
 * admitted requests run concurrently on their slots' streams, so a request
 * that arrives while others are on the GPU starts without waiting for them.
 * The server owns its own context (twiddle tables stay on the device) and a
 * scheduler thread; its functions may be called from any thread.
 */
typedef struct pa_server pa_server;

typedef struct pa_server_opts {
    uint64_t hbm_budget;  /* device bytes for requests in flight */
    int slots;            /* requests on the device at once */
    uint64_t max_n;       /* largest block accepted (<= PA_MAX_N) */
} pa_server_opts;

typedef struct pa_server_stats {
    uint64_t completed, failed;
    uint64_t bits;            /* input bits of completed requests */
    uint64_t peak_inflight;   /* most requests on the device at once */
    uint64_t peak_bytes;      /* most budget bytes in use at once */
    double lat_p50_ms, lat_p99_ms, lat_mean_ms;   /* submit -> result ready */
    double wall_s;            /* first submit -> last completion */
} pa_server_stats;

/* key/out of a request are device pointers (no host staging). */
#define PA_SUBMIT_DEVICE 1

/* PA_EINVAL if the budget cannot hold one request of max_n bits. */
int pa_server_create(int device, const pa_server_opts *opts, pa_server **server);

/* Queue one request.  Host pointers by default: key (ceil(n/64) words) must
 * stay valid and out (ceil(m/64) words) untouched until the request is done.
 * With PA_SUBMIT_DEVICE both are device pointers, and the server's streams do
 * not wait for the caller's: the key and out must be complete (written, and
 * no longer read or written by queued work) when the call is made.
 * *ticket identifies it. */
int pa_server_submit(pa_server *s, const uint64_t *key, uint64_t seed_a, uint64_t seed_b,
                     uint64_t n, uint64_t m, uint64_t *out, int flags, uint64_t *ticket);

/* The same for a device request whose key or out are still being produced by
 * queued work: `ready` (a hipEvent_t recorded after that work) is waited on by
 * the request's stream before its first kernel.  The event must stay valid
 * until the request is done.  NULL behaves as pa_server_submit; a non-NULL
 * event without PA_SUBMIT_DEVICE is PA_EINVAL. */
int pa_server_submit_after(pa_server *s, const uint64_t *key, uint64_t seed_a, uint64_t seed_b,
                           uint64_t n, uint64_t m, uint64_t *out, int flags, void *ready,
                           uint64_t *ticket);

/* Block until the request is done; its status and submit-to-result latency.
 * The ticket is then retired: a second wait on it returns PA_EINVAL.  Tickets
 * never waited on are kept until pa_server_destroy. */
int pa_server_wait(pa_server *s, uint64_t ticket, int *status, double *latency_ms);

/* Block until every request submitted so far is done. */
int pa_server_drain(pa_server *s);

/* Counts and latency percentiles over every request completed so far (the
 * server keeps one latency per completed request for them). */
int pa_server_get_stats(pa_server *s, pa_server_stats *stats);

/*
 * Open-loop load: submit jobs[i] (key/out/seeds/n/m) at arrival_s[i] seconds
 * after the call starts, from the calling thread, then wait for all.
 * latency_ms[i] and status[i] (either may be NULL) receive each request's
 * submit-to-result latency (-1 if it was not submitted) and status; a job
 * with c or d set is not submitted and gets PA_EINVAL.
 */
int pa_server_run_trace(pa_server *s, const pa_job *jobs, const double *arrival_s, size_t count,
                        int flags, double *latency_ms, int *status);

/* Finish what was submitted, then release everything. */
void pa_server_destroy(pa_server *s);

/* Size the workspace for blocks of up to n_max bits now. */
int pa_reserve(pa_ctx *ctx, uint64_t n_max);

/* Device bytes the workspace needs for one block of n bits. */
uint64_t pa_workspace_bytes(uint64_t n);

/*
 * Transform schedule.  A length-L transform is a few passes over the spectrum:
 * strided passes, then one contiguous pass whose tiles of 2^tile_log residues
 * are transformed whole in LDS.  Strided passes use tiles of 2^strided_tile_log
 * residues; for L = 3 * 2^k the first strided pass has 3 * 2^rows3_log rows
 * (and tiles of 3 * 2^(strided_tile_log - 2)).  Every geometry gives the same
 * (exact) result; they differ only in speed.  This is the counterpart of
 * matching the multiplication method to the operand size, which the paper
 * leaves to GMP (Sections 2.3 and 3.2.2).
 */
typedef struct pa_plan {
    int tile_log;          /* contiguous pass tile, log2 residues (<= 14) */
    int strided_tile_log;  /* strided pass tiles, log2 residues (0 with one pass) */
    int rows3_log;         /* lengths 3 * 2^k: log2 of the factor-3 pass rows / 3; else 0 */
    int passes;            /* out: passes per transform */
    float ms;              /* out: pa_tune, one hash of the tuning block with this plan;
                              pa_batch_group, one run of the group alone after
                              pa_batch_tune (0 before) */
} pa_plan;

/* Valid distinct geometries for blocks of n bits (the default first); writes
 * up to max, returns the count.  No device needed. */
int pa_plan_candidates(uint64_t n, pa_plan *out, int max);

/* The geometry ctx uses for blocks of n bits. */
int pa_plan_get(pa_ctx *ctx, uint64_t n, pa_plan *out);

/* Use geometry *p for every block whose transform length equals that of n
 * bits (passes and ms are ignored); NULL restores the default.  PA_EINVAL if
 * the geometry is not valid for that length.  A pa_mul made earlier keeps the
 * geometry it was made with. */
int pa_plan_set(pa_ctx *ctx, uint64_t n, const pa_plan *p);

/*
 * Autotune: time one hash of a seeded n-bit block (m = n / 2) reps times with
 * every candidate geometry of that transform length on the device, keep the
 * fastest for ctx (as pa_plan_set would) and return it in *best (may be NULL).
 * It first runs the default geometry for about 30 ms, so that the clocks have
 * risen, then sweeps the candidates twice (the second time in reverse order)
 * and keeps each one's faster time.  Allocates two temporary device buffers;
 * synchronises the context's stream.
 */
int pa_tune(pa_ctx *ctx, uint64_t n, int reps, pa_plan *best);

/*
 * Autotune a grouped batch: for every length group, time reps runs of the
 * group alone with each candidate geometry of its length (pa_plan_candidates;
 * two sweeps, the second in reverse order, after about 30 ms of whole-batch
 * runs so that the clocks have risen) and keep the fastest for that group.
 * Synchronises the context's stream and drops a recorded graph (call
 * pa_batch_capture again).  Every geometry computes the same bits.
 */
int pa_batch_tune(pa_batch *batch, int reps);

/* The batch's length groups: their number, and group i's transform length,
 * block count and geometry. */
size_t pa_batch_groups(const pa_batch *batch);
int pa_batch_group(const pa_batch *batch, size_t i, uint64_t *length, uint32_t *blocks,
                   pa_plan *plan);

/* Transform length used for a block of n bits (0 for n == 0 or n > PA_MAX_N).
 * The block takes the digit layout with less transform work (primes x L x
 * log2 L): W = 2 (64-bit digits, five primes) or W = 3 (96-bit digits, seven
 * primes, only for lengths that divide 3 * 2^22).  For D = ceil(n / (32 W))
 * digits, L is the smallest 2^k (k >= 6) or, when 3 * 2^(k-2) >= 2^18, the
 * smaller 3 * 2^(k-2), that is >= 2 D - 1 (a linear convolution's length). */
uint64_t pa_transform_length(uint64_t n);

/*
 * Toeplitz-hash variant: the family that the paper's Introduction names as the
 * usual privacy-amplification choice and the alternative to G_{c,d}, computed
 * on the same transform engine for a same-GPU comparison.  The member for t
 * (n + m - 1 random bits, the matrix's first column and row) is the m x n
 * matrix over GF(2) that is constant along its diagonals:
 *
 *     T[i][j] = t[i - j + n - 1],     y = T x,
 *     y_i = XOR_{j < n} (t[i + n - 1 - j] AND x_j),   0 <= i < m,
 *
 * i.e. y_i is the parity of coefficient i + n - 1 of the integer convolution
 * of the bit sequences t and x; the kernels compute that convolution exactly
 * with one element per bit over one prime, cutting the key into column pieces
 * when n + m - 1 exceeds the longest transform (3 * 2^25), and XOR the pieces.
 * Bit layout as above: key ceil(n/64) words, t ceil((n+m-1)/64) words, out
 * ceil(m/64) words, output bit i is y_i, bits past m in the top word are 0.
 * A NULL t draws t from seed_t: word i of t is the i-th SplitMix64(seed_t)
 * output (t is the stream of seed_t masked to n + m - 1 bits).
 * Sizes: 1 <= m <= n <= PA_MAX_N and m <= PA_TOEPLITZ_MAX_M, else PA_EINVAL.
 */
#define PA_TOEPLITZ_MAX_M ((uint64_t)3 << 24)

/* Synchronous: key, t (may be NULL: seeded) and out in host memory. */
int pa_toeplitz(pa_ctx *ctx, const uint64_t *key, const uint64_t *t, uint64_t seed_t,
                uint64_t n, uint64_t m, uint64_t *out);

/*
 * Asynchronous: d_key, d_t (may be NULL: seeded) and d_out are device
 * pointers; the work is queued on `stream` and the call returns at once.  It
 * shares the context's workspace with the other entry points, so calls on one
 * context must be ordered.
 */
int pa_toeplitz_async(pa_ctx *ctx, const uint64_t *d_key, const uint64_t *d_t, uint64_t seed_t,
                      uint64_t n, uint64_t m, uint64_t *d_out, void *stream);

/* Transform length of each piece for a Toeplitz block (0 if the sizes are out
 * of range); *pieces (may be NULL) receives the number of key pieces. */
uint64_t pa_toeplitz_length(uint64_t n, uint64_t m, uint64_t *pieces);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
