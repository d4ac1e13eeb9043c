// libpa runtime: device context, twiddle tables, plan and workspace, C ABI.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "context.h"
#include "persist.h"

using namespace pa;

namespace {

// ---------------------------------------------------------------------------
// host arithmetic for the tables
// ---------------------------------------------------------------------------

uint64_t hpow(uint64_t b, uint64_t e, uint64_t p)
{
    uint64_t r = 1;
    b %= p;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    return r;
}

uint32_t hmont(uint64_t x, uint64_t p) { return (uint32_t)(((x % p) << 32) % p); }
uint32_t hshoup(uint64_t w, uint64_t p) { return (uint32_t)((w << 32) / p); }

int fail(pa_ctx* ctx, int code, const char* what, hipError_t e = hipSuccess)
{
    if (ctx) {
        if (e != hipSuccess)
            snprintf(ctx->err, sizeof ctx->err, "%s: %s", what, hipGetErrorString(e));
        else
            snprintf(ctx->err, sizeof ctx->err, "%s", what);
    }
    return code;
}

#define PA_HIP(ctx, call)                                                        \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) return fail((ctx), PA_EDEVICE, #call, e_);         \
    } while (0)

// The context's HBM budget: may it replace `freed` bytes it holds by `added`?
int budget_check(pa_ctx* ctx, uint64_t freed, uint64_t added, const char* what)
{
    if (ctx->budget && ctx->held - freed + added > ctx->budget) {
        snprintf(ctx->err, sizeof ctx->err,
                 "%s: %llu device bytes would exceed the context's budget of %llu (holding %llu)",
                 what, (unsigned long long)added, (unsigned long long)ctx->budget,
                 (unsigned long long)(ctx->held - freed));
        return PA_ENOMEM;
    }
    return PA_OK;
}

uint64_t words_of(uint64_t bits) { return (bits + 63) / 64; }
uint64_t digits_of(uint64_t bits) { return (bits + 31) / 32; }
// Transform elements of an n-bit operand cut into digits of W 32-bit words.
uint64_t coeffs_of(uint64_t bits, int W) { return (bits + 32ull * W - 1) / (32ull * W); }

// Transform length for a block of n bits cut into D = ceil(n / 32 W) digits:
// the smallest L >= 2D - 1 among 2^l and, for long transforms, 3 * 2^(l-2) (a
// quarter shorter when it fits, as for n = 10^8 with 64-bit digits:
// 2D - 1 = 3 124 999 <= 3 * 2^20).
#ifndef PA_MIXED_RADIX_MIN_LOG
#define PA_MIXED_RADIX_MIN_LOG 18
#endif
// k = l - 2 >= kTileLog + 2 leaves the factor-3 pass at least 2 row bits.
static_assert(PA_MIXED_RADIX_MIN_LOG >= kTileLog + 4, "factor-3 pass needs a strided head");

struct Len {
    int f;       // 1 or 3
    int k;       // L = f 2^k
    int W = 2;   // digit words: 2 (64-bit digits, five primes) or 3 (96-bit, seven)
    uint64_t L() const { return (uint64_t)f << k; }
    int primes() const { return 2 * W + 1; }
};

// Smallest transform length >= need (at least 64).
Len len_for(uint64_t need)
{
    int l = 6;
    while ((1ull << l) < need) ++l;
    if (l >= PA_MIXED_RADIX_MIN_LOG && (3ull << (l - 2)) >= need) return {3, l - 2};
    return {1, l};
}

// Layout and length for an n-bit block: of 64-bit digits over five primes and
// 96-bit digits over seven, the one with less transform work, primes x L x
// log2 L (96-bit digits only for lengths that divide 3 2^22).  At
// n = 10^8: 5 x 3 2^20 against 7 x 2^21, the second; at 10^6: 5 x 2^15 against
// 7 x 2^15, the first.
Len plan_len(uint64_t n)
{
    Len a = len_for(2 * coeffs_of(n, 2) - 1);
    Len b = len_for(2 * coeffs_of(n, 3) - 1);
    b.W = 3;
    if (kOrder96 % b.L() != 0) return a;
    auto work = [](const Len& x) {
        return (double)x.primes() * (double)x.L() * (x.k + (x.f == 3 ? 1.585 : 0.0));
    };
    return work(b) < work(a) ? b : a;
}

uint64_t len_of(uint64_t n) { return plan_len(n).L(); }

// Residues per spectrum array (all primes) of an n-bit block.
uint64_t arr_elems(uint64_t n)
{
    const Len len = plan_len(n);
    return (uint64_t)len.primes() * len.L();
}

// Blocks with equal keys share every launch of a batch group.
uint64_t layout_key(uint64_t n)
{
    const Len len = plan_len(n);
    return (len.L() << 2) | (uint64_t)len.W;
}

// Coefficients of the chunks the carry apply kernel resolves for an n-bit
// block with an m-bit output: those that hold an output word's first bit
// (chunks wholly below bit n - m return at once).
uint64_t window_coeffs(uint64_t n, uint64_t m, int W)
{
    const uint64_t D = (n + 31) / 32;
    const uint64_t chunk = (uint64_t)kCarryThreads * carry_digits_per_thread((uint32_t)D, W);
    const uint64_t skipped = ((n - m) / 32 / chunk) * chunk / W;
    const uint64_t total = coeffs_of(n, W);
    return skipped < total ? total - skipped : 0;
}

uint32_t chunks_of(uint64_t D, int W)
{
    const uint64_t chunk = (uint64_t)kCarryThreads * carry_digits_per_thread((uint32_t)D, W);
    return (uint32_t)((D + chunk - 1) / chunk);
}

// Carry state words for the largest chunk count of any block up to D digits.
uint64_t status_words(uint64_t D) { return 2 * ((D + kCarryThreads * 4 - 1) / (kCarryThreads * 4)); }

#ifndef PA_TILE_SLACK
#define PA_TILE_SLACK 8
#endif
constexpr int kTileDefaultLog = 12;

// Default contiguous tile (log2 residues) for a transform of about 2^l
// residues run for `blocks` blocks at once.  Tiles of 2^12 (16 KB of LDS,
// three radix-16 steps) leave occupancy to the register budget (seven
// workgroups of four waves per CU) and keep the last wave of workgroups
// short; a lone short transform takes smaller tiles so that it still spreads
// over the chip.  pa_tune measures instead of guessing.
int plan_tile(int l, unsigned blocks = 1)
{
    if (l <= kTileMinLog) return l;
    int t = blocks >= 16 ? l : l - PA_TILE_SLACK;
    if (t < kTileMinLog) t = kTileMinLog;
    if (t > kTileDefaultLog) t = kTileDefaultLog;
    return t;
}

// Passes of a length-2^l transform: strided passes of at most 2^9 rows (each
// tile 2^ts residues, at least 4 columns), then one contiguous pass over whole
// tiles of 2^t.
int plan_passes(int l, int t, int ts, int* r)
{
    if (l <= t) {
        r[0] = l;
        return 1;
    }
    const int head = l - t;
    const int maxr = (ts - 2 < kStridedMaxLog) ? ts - 2 : kStridedMaxLog;
    const int k = (head + maxr - 1) / maxr;
    for (int i = 0; i < k; ++i)
        r[i] = head / k + (i < head % k ? 1 : 0);
    r[k] = t;
    return k + 1;
}

// Register steps of a length-2^r in-tile transform: radix up to 16.  Larger
// register radices need more vector registers per lane (radix 32: 94, five
// waves per SIMD; radix 16: 68, seven) and the occupancy is worth more than
// the saved LDS round trips (measured).
// The contiguous pass splits greedily (its last step has no twiddles, so a
// small last radix is cheap); strided passes split evenly, since every one of
// their steps carries twiddles and a lopsided split leaves threads idle.
int plan_steps(int r, int* st, bool strided)
{
    // A contiguous tile of at most 2^10 residues has at most 64 radix-16 DFTs
    // per step, one wave of its workgroup: radix 8 keeps two busy (measured 3%
    // faster at n = 10^6).
    const int rmax = (!strided && r <= 10) ? 3 : 4;
    const int k = (r + rmax - 1) / rmax;
    if (strided) {
        for (int i = 0; i < k; ++i) st[i] = r / k + (i < r % k ? 1 : 0);
        return k;
    }
    int n = 0;
    while (r > rmax) {
        st[n++] = rmax;
        r -= rmax;
    }
    st[n++] = r;
    return n;
}

uint64_t workspace_bytes_of(uint64_t elems, uint64_t D)
{
    return elems ? 2 * elems * 4 + std::max<uint64_t>(status_words(D), 1) * 4 : 0;
}

void free_workspace(pa_ctx* ctx)
{
    (void)hipFree(ctx->A);
    (void)hipFree(ctx->B);
    (void)hipFree(ctx->status);
    ctx->held -= workspace_bytes_of(ctx->cap_L, ctx->cap_D);
    ctx->A = ctx->B = ctx->status = nullptr;
    ctx->cap_L = ctx->cap_D = 0;
}

// Grow the workspace to two arrays of `elems` residues and the carry state of
// D digits, keeping any larger capacity it already has.
int ensure_caps(pa_ctx* ctx, uint64_t elems, uint64_t D)
{
    if (elems <= ctx->cap_L && D <= ctx->cap_D)
        return PA_OK;
    elems = std::max(elems, ctx->cap_L);
    D = std::max(D, ctx->cap_D);
    int rc = budget_check(ctx, workspace_bytes_of(ctx->cap_L, ctx->cap_D),
                          workspace_bytes_of(elems, D), "workspace");
    if (rc) return rc;
    PA_HIP(ctx, hipDeviceSynchronize());
    free_workspace(ctx);
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&ctx->A, elems * sizeof(uint32_t))) != hipSuccess ||
        (e = hipMalloc(&ctx->B, elems * sizeof(uint32_t))) != hipSuccess ||
        (e = hipMalloc(&ctx->status, std::max<uint64_t>(status_words(D), 1) * sizeof(uint32_t))) != hipSuccess) {
        free_workspace(ctx);
        return fail(ctx, PA_ENOMEM, "workspace allocation", e);
    }
    ctx->cap_L = elems;
    ctx->cap_D = D;
    ctx->held += workspace_bytes_of(elems, D);
    return PA_OK;
}

int ensure_workspace(pa_ctx* ctx, uint64_t n) { return ensure_caps(ctx, arr_elems(n), digits_of(n)); }

int ensure_staging(pa_ctx* ctx, uint64_t words, bool operands)
{
    if (words <= ctx->cap_words && (!operands || ctx->d_c))
        return PA_OK;
    // operand buffers, once made, are kept when the buffers grow
    const bool ops = operands || ctx->d_c != nullptr;
    const uint64_t w = words > ctx->cap_words ? words : ctx->cap_words;
    const uint64_t old_bytes = ctx->cap_words * 8 * (ctx->d_c ? 4 : 2);
    const uint64_t new_bytes = w * 8 * (ops ? 4 : 2);
    int rc = budget_check(ctx, old_bytes, new_bytes, "staging buffers");
    if (rc) return rc;
    if (ctx->cap_words) PA_HIP(ctx, hipDeviceSynchronize());   // nothing may still use them
    (void)hipFree(ctx->d_key);
    (void)hipFree(ctx->d_out);
    (void)hipFree(ctx->d_c);
    (void)hipFree(ctx->d_d);
    ctx->d_key = ctx->d_out = ctx->d_c = ctx->d_d = nullptr;
    ctx->cap_words = 0;
    ctx->held -= old_bytes;
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&ctx->d_key, w * 8)) != hipSuccess ||
        (e = hipMalloc(&ctx->d_out, w * 8)) != hipSuccess ||
        (ops && (e = hipMalloc(&ctx->d_c, w * 8)) != hipSuccess) ||
        (ops && (e = hipMalloc(&ctx->d_d, w * 8)) != hipSuccess)) {
        (void)hipFree(ctx->d_key);
        (void)hipFree(ctx->d_out);
        (void)hipFree(ctx->d_c);
        (void)hipFree(ctx->d_d);
        ctx->d_key = ctx->d_out = ctx->d_c = ctx->d_d = nullptr;
        return fail(ctx, PA_ENOMEM, "staging allocation", e);
    }
    ctx->cap_words = w;
    ctx->held += new_bytes;
    return PA_OK;
}

int check_sizes(pa_ctx* ctx, uint64_t n, uint64_t m)
{
    if (!ctx) return PA_EINVAL;
    if (n == 0 || m == 0 || m > n) return fail(ctx, PA_EINVAL, "need 1 <= m <= n");
    if (n > PA_MAX_N) return fail(ctx, PA_EINVAL, "n exceeds PA_MAX_N");
    return PA_OK;
}

// Optional per-launch timing for pa_hash_profile: each launch gets an event
// pair that its own dispatch stamps (no packets between the kernels).
struct Recorder {
    pa_ctx* ctx;
    pa_profile* prof;
    hipStream_t stream;
    hipError_t next(int kind, uint64_t bytes, LaunchEvents* ev)
    {
        const int i = prof->count;
        if (i >= PA_PROFILE_MAX) return hipErrorInvalidValue;
        prof->kind[i] = kind;
        prof->bytes[i] = bytes;
        prof->count = i + 1;
        ev->start = ctx->ev[2 * i];
        ev->stop = ctx->ev[2 * i + 1];
        return hipSuccess;
    }
};

// Launch `call`, which names the event pair ev_ (empty unless profiling).
#define PA_LAUNCH(ctx, rec, kind, bytes, call)                                   \
    do {                                                                         \
        LaunchEvents ev_{};                                                      \
        if (rec) PA_HIP(ctx, (rec)->next((kind), (bytes), &ev_));                \
        PA_HIP(ctx, call);                                                       \
    } while (0)

// Transform plan for L = f 2^k: tile size, passes, register steps, output scale.
struct Plan {
    int f = 1, k = 0, t = 0, ts = 0, P = 0;
    int W = 2;                         // digit words: 2W + 1 primes
    uint64_t L = 0;
    int r[8] = {}, s[8] = {}, logC[8] = {};
    int nsteps[8] = {};
    int steps[8][kMaxSteps] = {};
    uint32_t scale_w[kNumPrimes] = {}, scale_q[kNumPrimes] = {};
};

// Plan geometry: contiguous tile 2^t, strided tiles 2^ts (3 2^(ts-2) for the
// factor-3 pass, which has 3 2^r0 rows).  Zero fields take the defaults.
struct PlanParams {
    int t = 0, ts = 0, r0 = 0;
};

bool make_plan(Len len, Plan* pl, unsigned blocks = 1, PlanParams pp = {})
{
    pl->f = len.f;
    pl->k = len.k;
    pl->W = len.W;
    pl->L = len.L();
    const int t = pp.t ? pp.t : plan_tile(len.k + (len.f == 3 ? 2 : 0), blocks);
    // strided tiles: one size up for the factor-3 pass of long transforms
    // (3 2^9 rows of 8 columns at 2^12 contiguous tiles), else as contiguous
    const int ts = pp.ts ? pp.ts : ((len.f == 3 && t >= kTileDefaultLog) ? t + 1 : t);
    if (t > kTileLog || ts > kTileLog || ts < 6 || t < 1) return false;
    pl->t = t;
    pl->ts = ts;
    if (len.f == 1) {
        pl->P = plan_passes(len.k, t, ts, pl->r);
    } else {
        // the first strided pass carries the factor 3: 3 2^r0 rows, tiles of
        // 3 2^(ts-2) residues; the rest of the head as power-of-two passes
        const int head = len.k - t;
        if (head < 2) return false;
        const int r0 = pp.r0 ? pp.r0 : std::min(head, std::min(kStridedMaxLog, ts - 4));
        if (r0 < 2 || r0 > head || r0 > kStridedMaxLog) return false;
        pl->r[0] = r0;
        const int rest = head - r0;
        int P = 1;
        if (rest > 0) {
            const int maxr = (ts - 2 < kStridedMaxLog) ? ts - 2 : kStridedMaxLog;
            const int kk = (rest + maxr - 1) / maxr;
            if (kk + 2 > 8) return false;
            for (int i = 0; i < kk; ++i) pl->r[P++] = rest / kk + (i < rest % kk ? 1 : 0);
        }
        pl->r[P++] = t;
        pl->P = P;
    }
    if (pl->P > 8) return false;
    int rem = len.k;
    for (int i = 0; i < pl->P; ++i) {
        rem -= pl->r[i];
        pl->s[i] = rem;
        const bool strided = i + 1 < pl->P;
        if (strided)
            pl->logC[i] = (i == 0 && len.f == 3) ? ts - 2 - pl->r[i] : ts - pl->r[i];
        else
            pl->logC[i] = 0;
        if (strided && (pl->logC[i] < 2 || pl->logC[i] > pl->s[i])) return false;
        pl->nsteps[i] = plan_steps(pl->r[i], pl->steps[i], strided);
        if (pl->nsteps[i] > kMaxSteps) return false;
    }
    // c-hat is scaled by 2^32 / L (on the digits its first pass reads) so that the Montgomery
    // pointwise product yields x-hat c-hat / L.
    for (int pi = 0; pi < kNumPrimes; ++pi) {
        const uint64_t p = kPrimes[pi];
        const uint64_t w = ((1ull << 32) % p) * hpow(pl->L % p, p - 2, p) % p;
        pl->scale_w[pi] = (uint32_t)w;
        pl->scale_q[pi] = hshoup(w, p);
    }
    return true;
}

// Index of a transform length in the context's table of chosen plans.
int len_slot(Len len) { return (len.W == 3 ? 64 : 0) + (len.f == 3 ? 32 : 0) + len.k; }

// The plan a context uses for length len: its tuned or set geometry, else the
// defaults.
bool plan_for(const pa_ctx* ctx, Len len, Plan* pl)
{
    const int i = len_slot(len);
    if (ctx && i < pa_ctx::kPlanSlots && ctx->plans[i].t) {
        const PlanParams pp{ctx->plans[i].t, ctx->plans[i].ts, ctx->plans[i].r0};
        if (make_plan(len, pl, 1, pp)) return true;
    }
    return make_plan(len, pl);
}

// Operands of one block.  In batch mode the kernels read them from the job
// table instead, and `key_bytes` / `coeffs` / `out_bytes` are batch totals
// used only for the profile's byte counts.
struct Work {
    const uint32_t* key = nullptr;     // key digits
    const uint32_t* c = nullptr;       // explicit c digits or null
    const uint32_t* d = nullptr;       // explicit d digits or null
    uint64_t seed_a = 0, seed_b = 0, n = 0, m = 0;
    uint32_t* A = nullptr;
    uint32_t* B = nullptr;
    uint32_t* carry = nullptr;
    uint32_t* sums = nullptr;          // the carry kernels' column sums (free after
                                       // the pointwise product: A's array, or the
                                       // context's when A is a cached multiplier)
    uint64_t* out = nullptr;
    // batch mode
    const JobDesc* jobs = nullptr;
    unsigned batch = 1;
    uint32_t chunks = 0;               // grid width of the carry kernels
    int per = 4;                       // carry digits per thread
    uint64_t key_bytes = 0, coeffs = 0, out_bytes = 0;
    uint64_t window = 0;               // coefficients the apply kernel reads
    bool have_chat = false;            // A already holds c-hat (cached multiplier)
    bool only_chat = false;            // transform c into A and stop
};

// Shape of pass i of plan pl in a's geometry fields.
void pass_geometry(PassArgs& a, const Plan& pl, int i)
{
    a.f = (i == 0) ? pl.f : 1;
    a.r = pl.r[i];
    a.s = pl.s[i];
    a.logC = pl.logC[i];
    a.nsteps = pl.nsteps[i];
    a.steps_code = a.above_code = 0;
    int above = 0;
    for (int k = 0; k < kMaxSteps; ++k) {
        a.steps[k] = pl.steps[i][k];
        if (k < pl.nsteps[i]) {
            a.steps_code |= (uint32_t)pl.steps[i][k] << (4 * k);
            a.above_code |= (uint32_t)above << (4 * k);
            above += pl.steps[i][k];
        }
    }
}

// The launches of a batch recorded for the persistent kernel instead of being
// launched: each with the launches it depends on (indices in `launches`) and
// its level, the longest dependency chain before it.
struct PersistBuild {
    std::vector<PersistLaunch> launches;
    std::vector<int> level;
    uint32_t lds = 0;              // dynamic LDS the largest item needs

    int add(const PersistLaunch& l, int dep0, int dep1)
    {
        PersistLaunch x = l;
        x.dep0 = dep0;
        x.dep1 = dep1;
        int lv = 0;
        if (dep0 >= 0) lv = std::max(lv, level[dep0] + 1);
        if (dep1 >= 0) lv = std::max(lv, level[dep1] + 1);
        launches.push_back(x);
        level.push_back(lv);
        return (int)launches.size() - 1;
    }
};

// Queue every kernel of the hash (or of one batch group) on `stream`, or, with
// `pb`, record them as launches of the persistent batch kernel.
int enqueue_plan(pa_ctx* ctx, const Plan& pl, const Work& w, hipStream_t stream,
                 Recorder* rec = nullptr, PersistBuild* pb = nullptr)
{
    const unsigned batch = w.batch;
    const uint64_t L = pl.L;
    const int NP = 2 * pl.W + 1;                           // primes of the layout
    const uint64_t arr = batch * NP * 4ull * L;            // residue arrays, all blocks
    const uint64_t outD = NP * 4ull * w.coeffs;            // product coefficients kept
    const int P = pl.P;

    PassArgs base{};
    base.num_digits = (uint32_t)digits_of(w.n);
    base.n = w.n;
    base.L = (uint32_t)L;
    base.tb = Tables{ctx->pass_lo, ctx->pass_hi};
    base.store_limit = (uint32_t)L;
    base.jobs = w.jobs;
    base.primes = NP;
    base.dwords = pl.W;
    auto geometry = [&](PassArgs& a, int i) { pass_geometry(a, pl, i); };
    const uint32_t limit = (uint32_t)((coeffs_of(w.n, pl.W) + 3) & ~3ull);
    // persistent recording: the launch as queue items, and the last launch
    // of the multiplier's and of the key's (then the product's) chain
    int prev_c = -1, prev_x = -1;
    auto persist_pass = [&](const PassArgs& a, unsigned z) {
        PersistLaunch l{};
        l.kind = kPersistPass;
        l.W = pl.W;
        const uint32_t N = ((uint32_t)a.f << a.r) << a.logC;
        l.gx = (uint32_t)(L / N);
        l.gy = (uint32_t)NP;
        l.gz = z;
        l.pass = a;
        pb->lds = std::max<uint32_t>(pb->lds, 4u * N);
        return l;
    };

    // The first passes of c and of x share their geometry and are independent:
    // one launch runs both (grid.z = 2), so each fills the other's last wave.
    const bool dual = !w.jobs && !w.have_chat && !w.only_chat && P >= 2 && w.c == nullptr;
    for (int i = 0; i < P && !w.have_chat; ++i) {          // c-hat
        PassArgs a = base;
        a.role = kRoleMul;
        a.data = w.A;
        geometry(a, i);
        a.mode = kForward;
        a.src = kSrcArray;
        if (i == 0) {
            if (w.c) {
                a.src = kSrcDigits;
                a.digits = w.c;
            } else {
                a.src = kSrcSeed;
                a.seed = w.seed_a;
            }
        }
        if (i == 0) {
            // c-hat's factor 2^32 / L (for the Montgomery pointwise product),
            // applied to c's digits as its first pass reads them: the
            // transform is linear, and half of the first pass's rows are zero
            a.scale_in = 1;
            for (int pi = 0; pi < kNumPrimes; ++pi) {
                a.scale_w[pi] = pl.scale_w[pi];
                a.scale_q[pi] = pl.scale_q[pi];
            }
        }
        uint64_t in = (i == 0) ? (w.c ? w.key_bytes : 0) : arr;
        uint64_t outb = arr;
        unsigned z = batch;
        if (i == 0 && dual) {
            a.dual = 1;
            a.other = w.B;
            a.digits = w.key;
            in += w.key_bytes;
            outb += arr;
            z = 2;
        }
        if (pb) {
            prev_c = pb->add(persist_pass(a, z), prev_c, -1);
            continue;
        }
        PA_LAUNCH(ctx, rec, PA_K_NTT_PASS, in + outb, launch_pass(a, stream, z, ev_));
    }
    if (w.only_chat) return PA_OK;
    for (int i = (dual ? 1 : 0); i < P; ++i) {              // x-hat, pointwise, last inverse pass
        PassArgs a = base;
        a.role = kRoleKey;
        a.data = w.B;
        geometry(a, i);
        a.mode = (i == P - 1) ? kFused : kForward;
        if (P == 1) {
            a.store_limit = limit;
            a.limit_to_digits = 1;
        }
        a.other = w.A;
        a.src = (i == 0) ? kSrcDigits : kSrcArray;
        a.digits = w.key;
        uint64_t in = (i == 0) ? w.key_bytes : arr, outb = arr;
        if (i == P - 1) {
            in += arr;
            if (P == 1) outb = outD;
        }
        if (pb) {
            // the fused pass also reads c-hat
            prev_x = pb->add(persist_pass(a, batch), prev_x, i == P - 1 ? prev_c : -1);
            continue;
        }
        PA_LAUNCH(ctx, rec, PA_K_NTT_PASS, in + outb, launch_pass(a, stream, batch, ev_));
    }
    for (int i = P - 2; i >= 0; --i) {                      // remaining inverse passes
        PassArgs a = base;
        a.role = kRoleInv;
        a.data = w.B;
        geometry(a, i);
        a.mode = kInverse;
        a.src = kSrcArray;
        if (i == 0) {
            a.store_limit = limit;
            a.limit_to_digits = 1;
        }
        if (pb) {
            prev_x = pb->add(persist_pass(a, batch), prev_x, -1);
            continue;
        }
        PA_LAUNCH(ctx, rec, PA_K_NTT_PASS, arr + (i == 0 ? outD : arr),
                  launch_pass(a, stream, batch, ev_));
    }
    CarryArgs ca{};
    ca.res = w.B;
    ca.L = (uint32_t)L;
    ca.dwords = pl.W;
    ca.num_digits = (uint32_t)digits_of(w.n);
    ca.n = w.n;
    ca.m = w.m;
    if (w.d) {
        ca.addend_src = kSrcDigits;
        ca.addend = w.d;
    } else {
        ca.addend_src = kSrcSeed;
        ca.seed = w.seed_b;
    }
    ca.chunks = w.chunks;
    ca.per = w.per;
    ca.desc = w.carry;
    ca.sums = w.sums;
    ca.out = w.out;
    ca.jobs = w.jobs;
    const uint64_t chunk_bytes = 4ull * w.chunks * batch;
    if (pb) {
        PersistLaunch l{};
        l.W = pl.W;
        l.gx = w.chunks;
        l.gy = 1;
        l.gz = batch;
        l.carry = ca;
        l.kind = kPersistCarryLocal;
        const int local = pb->add(l, prev_x, -1);
        l.kind = kPersistCarryApply;
        pb->add(l, local, -1);
        pb->lds = std::max(pb->lds, persist_carry_lds_bytes(pl.W));
        return PA_OK;
    }
    // the window's column sums: a low word per digit, a word of high bits per
    // thread; written by the local kernel, read by the apply kernel
    const uint64_t sums_bytes = 4ull * w.window * pl.W + 4ull * ((w.window * pl.W + w.per - 1) / w.per);
    PA_LAUNCH(ctx, rec, PA_K_CARRY_LOCAL, outD + chunk_bytes + sums_bytes,
              launch_carry_local(ca, stream, batch, ev_));
    PA_LAUNCH(ctx, rec, PA_K_CARRY_APPLY, sums_bytes + chunk_bytes + w.out_bytes,
              launch_carry_apply(ca, stream, batch, ev_));
    return PA_OK;
}

// Queue the hash of one block held in the context's workspace.  c_words /
// d_words select explicit operands (device memory); null means seeded.
int enqueue(pa_ctx* ctx, const uint64_t* d_key, const uint64_t* c_words, const uint64_t* d_words,
            uint64_t seed_a, uint64_t seed_b, uint64_t n, uint64_t m, uint64_t* d_out,
            hipStream_t stream, Recorder* rec = nullptr)
{
    int rc = ensure_workspace(ctx, n);
    if (rc) return rc;
    Plan pl;
    if (!plan_for(ctx, plan_len(n), &pl)) return fail(ctx, PA_EINVAL, "internal: bad pass plan");
    Work w;
    w.key = reinterpret_cast<const uint32_t*>(d_key);
    w.c = reinterpret_cast<const uint32_t*>(c_words);
    w.d = reinterpret_cast<const uint32_t*>(d_words);
    w.seed_a = seed_a;
    w.seed_b = seed_b;
    w.n = n;
    w.m = m;
    w.A = ctx->A;
    w.B = ctx->B;
    w.carry = ctx->status;
    w.sums = ctx->A;
    w.out = d_out;
    w.chunks = chunks_of(digits_of(n), pl.W);
    w.per = carry_digits_per_thread((uint32_t)digits_of(n), pl.W);
    w.key_bytes = (n + 7) / 8;
    w.coeffs = coeffs_of(n, pl.W);
    w.window = window_coeffs(n, m, pl.W);
    w.out_bytes = words_of(m) * 8;
    return enqueue_plan(ctx, pl, w, stream, rec);
}

}  // namespace

namespace pa {

uint64_t block_workspace_bytes(uint64_t n)
{
    return 2 * ((4ull * arr_elems(n) + 255) & ~255ull) + ((4ull * status_words(digits_of(n)) + 255) & ~255ull);
}

void block_layout(uint64_t n, uint8_t* base, BlockBufs* b)
{
    const uint64_t arr = (4ull * arr_elems(n) + 255) & ~255ull;
    b->A = reinterpret_cast<uint32_t*>(base);
    b->B = reinterpret_cast<uint32_t*>(base + arr);
    b->carry = reinterpret_cast<uint32_t*>(base + 2 * arr);
}

int enqueue_block(pa_ctx* ctx, const BlockBufs& b, hipStream_t stream)
{
    Plan pl;
    if (!plan_for(ctx, plan_len(b.n), &pl)) return fail(ctx, PA_EINVAL, "internal: bad pass plan");
    Work w;
    w.key = b.key;
    w.c = b.c;
    w.d = b.d;
    w.seed_a = b.seed_a;
    w.seed_b = b.seed_b;
    w.n = b.n;
    w.m = b.m;
    w.A = b.A;
    w.B = b.B;
    w.carry = b.carry;
    w.sums = b.A;
    w.out = b.out;
    w.chunks = chunks_of(digits_of(b.n), pl.W);
    w.per = carry_digits_per_thread((uint32_t)digits_of(b.n), pl.W);
    w.key_bytes = (b.n + 7) / 8;
    w.coeffs = coeffs_of(b.n, pl.W);
    w.window = window_coeffs(b.n, b.m, pl.W);
    w.out_bytes = words_of(b.m) * 8;
    return enqueue_plan(ctx, pl, w, stream);
}

int set_error(pa_ctx* ctx, int code, const char* what) { return fail(ctx, code, what); }

}  // namespace pa

namespace {

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (pa_hash_async_noalloc): the two
// spectra and the carry state of one block, in device memory that exists from
// the moment the library's code object is loaded on a GPU until the process
// ends.  In host code `scratch` is only a stand-in for the symbol, never a
// device address: each GPU holds its own copy, whose address hipGetSymbolAddress
// gives once per device (scratch_address, from pa_init), and only that address
// is ever passed to a kernel.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[PA_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// The device address of `device`'s copy of the scratch; that device must be
// current.  Taken on the first call for a device and kept.
int scratch_address(pa_ctx* ctx, int device, uint8_t** out)
{
    if (device < 0 || device >= kMaxDevices) return fail(ctx, PA_ENODEV, "device index too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(ctx, PA_EDEVICE, "hipGetSymbolAddress(scratch)", e);
        g_scratch[device] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch[device];
    return PA_OK;
}

}  // namespace

#ifndef PA_ENABLE_PERSISTENT
#define PA_ENABLE_PERSISTENT 0
#endif

struct pa_batch {
    pa_ctx* ctx = nullptr;
    int device = 0;      // for pa_batch_destroy, which may follow pa_destroy(ctx)
    struct Group {
        Plan plan;
        uint32_t first = 0, count = 0;   // range in the job table
        uint32_t chunks = 0;             // widest carry grid of the group
        int per = 4;
        uint64_t key_bytes = 0, coeffs = 0, out_bytes = 0, window = 0;
        float tuned_ms = 0.f;            // pa_batch_tune: one run of the group alone
    };
    std::vector<Group> groups;
    JobDesc* d_jobs = nullptr;
    uint8_t* ws = nullptr;
    uint64_t ws_bytes = 0;
    size_t valid = 0;
    size_t launches = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // persistent mode: the launch table, the queue counters, the grid, and the
    // abort flag of the last run copied to host memory
    int mode = PA_BATCH_GROUPED;
    PersistLaunch* d_launch = nullptr;
    uint32_t* d_ctr = nullptr;
    uint32_t* h_abort = nullptr;
    PersistArgs pargs{};
    uint32_t workgroups = 0, lds = 0;
    uint64_t table_bytes = 0;
};

namespace {

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Geometry of a batch group of `blocks` blocks of length len: the context's
// tuned or set geometry for that length, else the batch default (larger
// tiles when many blocks fill the device together).
bool batch_plan(const pa_ctx* ctx, Len len, unsigned blocks, Plan* pl)
{
    const int i = len_slot(len);
    if (i < pa_ctx::kPlanSlots && ctx->plans[i].t) {
        const PlanParams pp{ctx->plans[i].t, ctx->plans[i].ts, ctx->plans[i].r0};
        if (make_plan(len, pl, blocks, pp)) return true;
    }
    return make_plan(len, pl, blocks);
}

// Record every group's launches as queue items, order them by level (then as
// recorded: group by group, largest transforms first), number the items and
// the per-block done counters, and upload the table.
int build_persistent(pa_batch* b, const pa_batch_opts* opts)
{
    pa_ctx* ctx = b->ctx;
    PersistBuild pb;
    for (size_t gi = b->groups.size(); gi-- > 0;) {
        const auto& g = b->groups[gi];
        Work w;
        w.jobs = b->d_jobs + g.first;
        w.batch = g.count;
        w.chunks = g.chunks;
        w.per = g.per;
        int rc = enqueue_plan(ctx, g.plan, w, nullptr, nullptr, &pb);
        if (rc) return rc;
    }
    const size_t nl = pb.launches.size();
    std::vector<int> order(nl);
    for (size_t i = 0; i < nl; ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return pb.level[x] < pb.level[y]; });
    std::vector<int> pos(nl);
    for (size_t k = 0; k < nl; ++k) pos[order[k]] = (int)k;
    std::vector<PersistLaunch> table(nl);
    uint64_t items = 0, counters = 0;
    for (size_t k = 0; k < nl; ++k) {
        PersistLaunch l = pb.launches[order[k]];
        l.dep0 = l.dep0 >= 0 ? pos[l.dep0] : -1;
        l.dep1 = l.dep1 >= 0 ? pos[l.dep1] : -1;
        l.first = (uint32_t)items;
        l.ctr_base = (uint32_t)counters;
        items += (uint64_t)l.gx * l.gy * l.gz;
        counters += l.gz;
        table[k] = l;
    }
    if (items >= (1ull << 31) || counters >= (1ull << 28))
        return fail(ctx, PA_EINVAL, "batch too large for the persistent queue");
    b->lds = pb.lds;
    PA_HIP(ctx, persist_grid(b->lds, ctx->device, &b->workgroups));
    b->table_bytes = sizeof(PersistLaunch) * nl + 4ull * (kPersistCounters + counters);
    hipError_t e;
    if ((e = hipMalloc(&b->d_launch, sizeof(PersistLaunch) * nl)) != hipSuccess ||
        (e = hipMalloc(&b->d_ctr, 4ull * (kPersistCounters + counters))) != hipSuccess)
        return fail(ctx, PA_ENOMEM, "persistent batch table allocation", e);
    if ((e = hipHostMalloc((void**)&b->h_abort, sizeof(uint32_t), hipHostMallocDefault)) != hipSuccess)
        return fail(ctx, PA_ENOMEM, "pinned host flag", e);
    *b->h_abort = 0;
    PA_HIP(ctx, hipMemcpy(b->d_launch, table.data(), sizeof(PersistLaunch) * nl,
                          hipMemcpyHostToDevice));
    PersistArgs& a = b->pargs;
    a.launches = b->d_launch;
    a.nlaunch = (uint32_t)nl;
    a.total = (uint32_t)items;
    a.ctr = b->d_ctr;
    a.ncounters = (uint32_t)counters;
    // the wait bound in ticks of the device's constant-rate clock (kHz)
    int clock_khz = 0;
    PA_HIP(ctx, hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, ctx->device));
    const uint64_t wait_us = (opts && opts->wait_us) ? opts->wait_us : 2000000u;
    a.wait_ticks = wait_us * (uint64_t)(clock_khz > 0 ? clock_khz : 100000) / 1000u;
    a.force_abort = opts ? opts->force_abort : 0;
    return PA_OK;
}

// Groups are independent: they run concurrently on the context's side
// streams, forked from and joined back into `stream` with events (this also
// holds inside a graph capture, where it becomes parallel branches).
int enqueue_batch(pa_batch* b, hipStream_t stream)
{
    pa_ctx* ctx = b->ctx;
    if (b->mode == PA_BATCH_PERSISTENT) {
        PA_HIP(ctx, launch_persist(b->pargs, b->workgroups, b->lds, stream));
        PA_HIP(ctx, hipMemcpyAsync(b->h_abort, b->d_ctr + 1, sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, stream));
        return PA_OK;
    }
    const int ns = (int)std::min<size_t>(b->groups.size(), pa_ctx::kSide);
    if (ns > 1) {
        PA_HIP(ctx, hipEventRecord(ctx->fork, stream));
        for (int i = 0; i < ns; ++i) PA_HIP(ctx, hipStreamWaitEvent(ctx->side[i], ctx->fork, 0));
    }
    // largest transforms first, so the long groups start early
    for (size_t gi = b->groups.size(); gi-- > 0;) {
        const auto& g = b->groups[gi];
        const hipStream_t st = ns > 1 ? ctx->side[gi % ns] : stream;
        Work w;
        w.jobs = b->d_jobs + g.first;
        w.batch = g.count;
        w.chunks = g.chunks;
        w.per = g.per;
        w.key_bytes = g.key_bytes;
        w.coeffs = g.coeffs;
        w.window = g.window;
        w.out_bytes = g.out_bytes;
        int rc = enqueue_plan(ctx, g.plan, w, st);
        if (rc) return rc;
    }
    if (ns > 1) {
        for (int i = 0; i < ns; ++i) {
            PA_HIP(ctx, hipEventRecord(ctx->join[i], ctx->side[i]));
            PA_HIP(ctx, hipStreamWaitEvent(stream, ctx->join[i], 0));
        }
    }
    return PA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Toeplitz variant: y_i = (t * x)[i + n - 1] mod 2 on the transform passes, one
// element per bit over the first prime.  A block whose linear convolution is
// longer than the longest transform (kOrder) is cut into column pieces of the
// key: piece [j0, j0 + w) is itself a Toeplitz product of width w with the t
// bits [n - j0 - w, n - j0 + m - 1), and the pieces' outputs are XORed.
// ---------------------------------------------------------------------------
namespace {

struct ToeplitzPlan {
    uint64_t pieces = 0, width = 0;
    Len len{1, 6};
};

bool toeplitz_plan(uint64_t n, uint64_t m, ToeplitzPlan* tp)
{
    const uint64_t lmax = kOrder;
    if (n == 0 || m == 0 || m > n || n > PA_MAX_N || m > PA_TOEPLITZ_MAX_M) return false;
    const uint64_t wmax = lmax - m + 1;
    tp->pieces = (n + wmax - 1) / wmax;
    tp->width = (n + tp->pieces - 1) / tp->pieces;
    tp->len = len_for(tp->width + m - 1);
    return tp->len.L() <= lmax;
}

int enqueue_toeplitz(pa_ctx* ctx, const uint64_t* d_key, const uint64_t* d_t, uint64_t n,
                     uint64_t m, uint64_t* d_out, hipStream_t stream)
{
    ToeplitzPlan tp;
    if (!toeplitz_plan(n, m, &tp)) return fail(ctx, PA_EINVAL, "Toeplitz sizes out of range");
    Plan pl;
    if (!plan_for(ctx, tp.len, &pl)) return fail(ctx, PA_EINVAL, "internal: bad pass plan");
    const uint64_t L = pl.L;
    int rc = ensure_caps(ctx, L, 0);
    if (rc) return rc;
    const int P = pl.P;
    PassArgs base{};
    base.L = (uint32_t)L;
    base.tb = Tables{ctx->pass_lo, ctx->pass_hi};
    base.store_limit = (uint32_t)L;
    base.primes = 1;
    for (uint64_t piece = 0; piece < tp.pieces; ++piece) {
        const uint64_t j0 = piece * tp.width;
        const uint64_t w = std::min(tp.width, n - j0);
        const uint64_t need = w + m - 1;                   // convolution positions used
        const uint32_t limit = (uint32_t)((need + 3) & ~3ull);
        for (int i = 0; i < P; ++i) {                      // t-hat into A
            PassArgs a = base;
            pass_geometry(a, pl, i);
            a.data = ctx->A;
            a.mode = kForward;
            a.src = kSrcArray;
            if (i == 0) {
                a.src = kSrcBits;
                a.digits = reinterpret_cast<const uint32_t*>(d_t);
                a.bit_off = n - j0 - w;
                a.n = need;
                // t-hat's factor 2^32 / L, on its bits as they are read
                a.scale_in = 1;
                a.scale_w[0] = pl.scale_w[0];
                a.scale_q[0] = pl.scale_q[0];
            }
            PA_HIP(ctx, launch_pass(a, stream));
        }
        for (int i = 0; i < P; ++i) {                      // x-hat, pointwise, last inverse pass
            PassArgs a = base;
            pass_geometry(a, pl, i);
            a.data = ctx->B;
            a.other = ctx->A;
            a.mode = (i == P - 1) ? kFused : kForward;
            a.src = kSrcArray;
            if (i == 0) {
                a.src = kSrcBits;
                a.digits = reinterpret_cast<const uint32_t*>(d_key);
                a.bit_off = j0;
                a.n = w;
            }
            if (P == 1) a.store_limit = limit;
            PA_HIP(ctx, launch_pass(a, stream));
        }
        for (int i = P - 2; i >= 0; --i) {                 // remaining inverse passes
            PassArgs a = base;
            pass_geometry(a, pl, i);
            a.data = ctx->B;
            a.mode = kInverse;
            a.src = kSrcArray;
            if (i == 0) a.store_limit = limit;
            PA_HIP(ctx, launch_pass(a, stream));
        }
        PA_HIP(ctx, launch_parity(ctx->B, w - 1, m, d_out, piece > 0, stream));
    }
    return PA_OK;
}

// t drawn from seed_t into the context's buffer.
int seeded_t(pa_ctx* ctx, uint64_t seed_t, uint64_t bits, hipStream_t stream, const uint64_t** t)
{
    const uint64_t w = words_of(bits);
    if (w > ctx->cap_tbits) {
        int rc = budget_check(ctx, ctx->cap_tbits * 8, w * 8, "Toeplitz t buffer");
        if (rc) return rc;
        PA_HIP(ctx, hipDeviceSynchronize());
        (void)hipFree(ctx->tbits);
        ctx->held -= ctx->cap_tbits * 8;
        ctx->tbits = nullptr;
        ctx->cap_tbits = 0;
        hipError_t e = hipMalloc(&ctx->tbits, w * 8);
        if (e != hipSuccess) return fail(ctx, PA_ENOMEM, "Toeplitz t allocation", e);
        ctx->cap_tbits = w;
        ctx->held += w * 8;
    }
    PA_HIP(ctx, launch_stream_words(seed_t, w, ctx->tbits, stream));
    *t = ctx->tbits;
    return PA_OK;
}

int check_toeplitz(pa_ctx* ctx, uint64_t n, uint64_t m)
{
    if (!ctx) return PA_EINVAL;
    if (n == 0 || m == 0 || m > n) return fail(ctx, PA_EINVAL, "need 1 <= m <= n");
    if (n > PA_MAX_N) return fail(ctx, PA_EINVAL, "n exceeds PA_MAX_N");
    if (m > PA_TOEPLITZ_MAX_M) return fail(ctx, PA_EINVAL, "m exceeds PA_TOEPLITZ_MAX_M");
    return PA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan geometry choice: explicit, or timed on the device (pa_tune)
// ---------------------------------------------------------------------------
namespace {

bool same_plan(const Plan& a, const Plan& b)
{
    if (a.P != b.P) return false;
    for (int i = 0; i < a.P; ++i) {
        if (a.r[i] != b.r[i] || a.logC[i] != b.logC[i] || a.nsteps[i] != b.nsteps[i]) return false;
        for (int k = 0; k < a.nsteps[i]; ++k)
            if (a.steps[i][k] != b.steps[i][k]) return false;
    }
    return true;
}

void describe(const Plan& pl, pa_plan* out)
{
    out->tile_log = pl.t;
    out->strided_tile_log = pl.P > 1 ? pl.ts : 0;
    out->rows3_log = pl.f == 3 ? pl.r[0] : 0;
    out->passes = pl.P;
    out->ms = 0.f;
}

// Distinct valid geometries for length len: the default first, then those
// with at most one pass more than the fewest possible, fewest passes and
// largest tiles first.
int candidates(Len len, pa_plan* out, int max)
{
    constexpr int kMaxFound = 256;
    static thread_local Plan found[kMaxFound];
    int cnt = 0;
    Plan d;
    const bool have_default = make_plan(len, &d);
    if (have_default) found[cnt++] = d;
    const int tlo = std::min(len.k, 10);
    int min_p = have_default ? d.P : 99;
    for (int t = kTileLog; t >= tlo; --t)
        for (int ts = kTileLog; ts >= 10; --ts)
            for (int r0 = (len.f == 3 ? kStridedMaxLog : 0); r0 >= (len.f == 3 ? 2 : 0); --r0) {
                Plan pl;
                if (!make_plan(len, &pl, 1, PlanParams{t, ts, r0})) continue;
                bool dup = false;
                for (int i = 0; i < cnt && !dup; ++i) dup = same_plan(found[i], pl);
                if (dup || cnt >= kMaxFound) continue;
                found[cnt++] = pl;
                min_p = std::min(min_p, pl.P);
            }
    int order[kMaxFound];
    int k = 0;
    for (int i = 0; i < cnt; ++i)
        if (i == 0 && have_default) order[k++] = i;
    for (int P = min_p; P <= min_p + 1; ++P)
        for (int i = have_default ? 1 : 0; i < cnt; ++i)
            if (found[i].P == P) order[k++] = i;
    const int n = std::min(k, max);
    for (int i = 0; i < n; ++i) describe(found[order[i]], &out[i]);
    return n;
}

// The tuning cache: one line per tuned transform length,
//   pa_tune <arch> <W> <f> <k> <t> <ts> <r0> <ms>
// (digit words, L = f 2^k, the geometry, the measured time of one hash).
// Later lines override earlier ones; lines for another architecture, of
// another format or with a geometry invalid for their length are ignored.
bool append_tuned(const char* path, const char* arch, Len len, int t, int ts, int r0, float ms)
{
    FILE* f = fopen(path, "a");
    if (!f) return false;
    const int ok = fprintf(f, "pa_tune %s %d %d %d %d %d %d %.6f\n", arch, len.W, len.f, len.k, t,
                           ts, r0, (double)ms);
    return fclose(f) == 0 && ok > 0;
}

// Load the cache into ctx->plans; a missing file is an empty cache.
int load_tuned(pa_ctx* ctx)
{
    FILE* f = fopen(ctx->tune_cache, "r");
    if (!f) return PA_OK;
    char line[256], arch[64];
    while (fgets(line, sizeof line, f)) {
        int W = 0, fct = 0, k = 0, t = 0, ts = 0, r0 = 0;
        float ms = 0.f;
        if (sscanf(line, "pa_tune %63s %d %d %d %d %d %d %f", arch, &W, &fct, &k, &t, &ts, &r0, &ms) != 8)
            continue;
        if (strcmp(arch, ctx->arch) != 0 || (W != 2 && W != 3) || (fct != 1 && fct != 3) || k < 6 ||
            k > kLogMaxLen)
            continue;
        Len len{fct, k};
        len.W = W;
        Plan pl;
        if (!make_plan(len, &pl, 1, PlanParams{t, ts, r0})) continue;
        const int slot = len_slot(len);
        if (slot < pa_ctx::kPlanSlots) ctx->plans[slot] = pa_ctx::PlanChoice{t, ts, r0};
    }
    const bool bad = ferror(f);
    fclose(f);
    return bad ? fail(ctx, PA_EIO, "reading the tuning cache file") : PA_OK;
}

}  // namespace

extern "C" {

const char* pa_strerror(int status)
{
    switch (status) {
    case PA_OK: return "ok";
    case PA_EINVAL: return "invalid argument";
    case PA_ENOMEM: return "out of memory";
    case PA_EDEVICE: return "device error";
    case PA_ENODEV: return "no usable gfx950 device";
    case PA_EIO: return "tuning cache file error";
    default: return "unknown status";
    }
}

const char* pa_last_error(const pa_ctx* ctx) { return ctx ? ctx->err : ""; }

uint64_t pa_transform_length(uint64_t n)
{
    if (n == 0 || n > PA_MAX_N) return 0;
    return len_of(n);
}

uint64_t pa_ctx_bytes(const pa_ctx* ctx) { return ctx ? ctx->held : 0; }

uint64_t pa_workspace_bytes(uint64_t n)
{
    if (n == 0 || n > PA_MAX_N) return 0;
    const uint64_t D = digits_of(n);
    return 2 * arr_elems(n) * 4 + status_words(D) * 4;
}

int pa_init(pa_ctx** out, int device, const pa_opts* opts)
{
    if (!out) return PA_EINVAL;
    *out = nullptr;
    if (opts && opts->tune_cache && strlen(opts->tune_cache) >= sizeof(((pa_ctx*)nullptr)->tune_cache))
        return PA_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return PA_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PA_ENODEV;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PA_ENODEV;

    pa_ctx* ctx = new (std::nothrow) pa_ctx;
    if (!ctx) return PA_ENOMEM;
    ctx->device = device;
    snprintf(ctx->arch, sizeof ctx->arch, "%s", prop.gcnArchName);
    if (char* colon = strchr(ctx->arch, ':')) *colon = 0;   // drop feature suffixes
    if (opts) {
        ctx->budget = opts->hbm_budget;
        if (opts->tune_cache) snprintf(ctx->tune_cache, sizeof ctx->tune_cache, "%s", opts->tune_cache);
    }
    int rc = PA_OK;
    uint32_t *h_lo = nullptr, *h_hi = nullptr;
    do {
        if (hipSetDevice(device) != hipSuccess) { rc = PA_ENODEV; break; }
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            rc = PA_EDEVICE;
            break;
        }
        bool ok = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; i < pa_ctx::kSide && ok; ++i)
            ok = hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&ctx->join[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            rc = PA_EDEVICE;
            break;
        }
        const uint64_t table_bytes = sizeof(uint32_t) * kNumPrimes * (4096 + kRootHi);
        if ((rc = budget_check(ctx, 0, table_bytes, "twiddle tables")) != PA_OK) break;
        h_lo = new (std::nothrow) uint32_t[kNumPrimes * 4096];
        h_hi = new (std::nothrow) uint32_t[kNumPrimes * kRootHi];
        if (!h_lo || !h_hi) { rc = PA_ENOMEM; break; }
        for (int pi = 0; pi < kNumPrimes; ++pi) {
            const uint64_t p = kPrimes[pi];
            // w^E for the order-3 2^25 root w; a prime whose root r has order
            // 3 2^22 stores r^(E / 8), defined for the multiples of 8 that
            // its transforms use (other low entries stay 0)
            const uint64_t wo = kRoot[pi];
            const int sh = kRootShift[pi];
            for (int i = 0; i < 4096; ++i)
                h_lo[pi * 4096 + i] = (i & ((1 << sh) - 1)) ? 0u : hmont(hpow(wo, (uint64_t)(i >> sh), p), p);
            const uint64_t step = hpow(wo, 4096u >> sh, p);
            uint64_t w = 1;
            for (int j = 0; j < kRootHi; ++j) {
                h_hi[pi * kRootHi + j] = hmont(w, p);
                w = w * step % p;
            }
        }
        if (hipMalloc(&ctx->pass_lo, sizeof(uint32_t) * kNumPrimes * 4096) != hipSuccess ||
            hipMalloc(&ctx->pass_hi, sizeof(uint32_t) * kNumPrimes * kRootHi) != hipSuccess) {
            rc = PA_ENOMEM;
            break;
        }
        ctx->held += table_bytes;
        if (hipMemcpy(ctx->pass_lo, h_lo, sizeof(uint32_t) * kNumPrimes * 4096,
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->pass_hi, h_hi, sizeof(uint32_t) * kNumPrimes * kRootHi,
                      hipMemcpyHostToDevice) != hipSuccess) {
            rc = PA_EDEVICE;
            break;
        }
        rc = scratch_address(ctx, device, &ctx->scratch);
        if (rc == PA_OK && ctx->tune_cache[0]) rc = load_tuned(ctx);
    } while (0);
    delete[] h_lo;
    delete[] h_hi;
    if (rc != PA_OK) {
        pa_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return PA_OK;
}

void pa_destroy(pa_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    // work queued on callers' streams (pa_hash_async and the like) may still
    // use the workspace and tables: wait for the whole device, not just ctx->stream
    (void)hipDeviceSynchronize();
    free_workspace(ctx);
    (void)hipFree(ctx->d_key);
    (void)hipFree(ctx->d_out);
    (void)hipFree(ctx->d_c);
    (void)hipFree(ctx->d_d);
    (void)hipFree(ctx->tbits);
    (void)hipFree(ctx->pass_lo);
    (void)hipFree(ctx->pass_hi);
    if (ctx->have_events)
        for (auto& e : ctx->ev) (void)hipEventDestroy(e);
    for (int i = 0; i < pa_ctx::kSide; ++i) {
        if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
        if (ctx->join[i]) (void)hipEventDestroy(ctx->join[i]);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int pa_reserve(pa_ctx* ctx, uint64_t n_max)
{
    int rc = check_sizes(ctx, n_max, 1);
    if (rc) return rc;
    PA_HIP(ctx, hipSetDevice(ctx->device));
    return ensure_workspace(ctx, n_max);
}

int pa_hash_async(pa_ctx* ctx, const uint64_t* d_key, uint64_t seed_a, uint64_t seed_b,
                  uint64_t n, uint64_t m, uint64_t* d_out, void* stream)
{
    int rc = check_sizes(ctx, n, m);
    if (rc) return rc;
    if (!d_key || !d_out) return fail(ctx, PA_EINVAL, "null key or output pointer");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    return enqueue(ctx, d_key, nullptr, nullptr, seed_a, seed_b, n, m, d_out,
                   (hipStream_t)stream);
}

int pa_hash_async_noalloc(pa_ctx* ctx, const uint64_t* d_key, uint64_t seed_a, uint64_t seed_b,
                          uint64_t n, uint64_t m, uint64_t* d_out, void* stream)
{
    int rc = check_sizes(ctx, n, m);
    if (rc) return rc;
    if (!d_key || !d_out) return fail(ctx, PA_EINVAL, "null key or output pointer");
    const uint64_t need = block_workspace_bytes(n);
    if (need > PA_NOALLOC_MAX_BYTES) {
        char what[160];
        snprintf(what, sizeof what,
                 "n = %llu needs %llu scratch bytes; the allocation-free entry point has "
                 "PA_NOALLOC_MAX_BYTES = %llu",
                 (unsigned long long)n, (unsigned long long)need,
                 (unsigned long long)PA_NOALLOC_MAX_BYTES);
        return fail(ctx, PA_EINVAL, what);
    }
    if (!ctx->scratch) return fail(ctx, PA_EDEVICE, "scratch address missing");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    // Nothing in the scratch must start at zero: the first forward pass writes
    // every residue of both spectra, and the carry kernels' first launch writes
    // every chunk's carry function before the second reads any.
    BlockBufs b;
    block_layout(n, ctx->scratch, &b);
    b.key = reinterpret_cast<const uint32_t*>(d_key);
    b.seed_a = seed_a;
    b.seed_b = seed_b;
    b.n = n;
    b.m = m;
    b.out = d_out;
    return enqueue_block(ctx, b, (hipStream_t)stream);
}

int pa_hash_profile(pa_ctx* ctx, const uint64_t* d_key, uint64_t seed_a, uint64_t seed_b,
                    uint64_t n, uint64_t m, uint64_t* d_out, void* stream, pa_profile* prof)
{
    int rc = check_sizes(ctx, n, m);
    if (rc) return rc;
    if (!d_key || !d_out || !prof) return fail(ctx, PA_EINVAL, "null pointer");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    if (!ctx->have_events) {
        for (auto& e : ctx->ev) PA_HIP(ctx, hipEventCreate(&e));
        ctx->have_events = true;
    }
    rc = ensure_workspace(ctx, n);
    if (rc) return rc;
    memset(prof, 0, sizeof *prof);
    Recorder rec{ctx, prof, (hipStream_t)stream};
    rc = enqueue(ctx, d_key, nullptr, nullptr, seed_a, seed_b, n, m, d_out, (hipStream_t)stream,
                 &rec);
    PA_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    if (rc) return rc;
    for (int i = 0; i < prof->count; ++i)
        PA_HIP(ctx, hipEventElapsedTime(&prof->ms[i], ctx->ev[2 * i], ctx->ev[2 * i + 1]));
    return PA_OK;
}

static int hash_host(pa_ctx* ctx, const uint64_t* key, const uint64_t* c, const uint64_t* d,
                     uint64_t seed_a, uint64_t seed_b, uint64_t n, uint64_t m, uint64_t* out)
{
    int rc = check_sizes(ctx, n, m);
    if (rc) return rc;
    if (!key || !out) return fail(ctx, PA_EINVAL, "null key or output pointer");
    const bool explicit_ops = c != nullptr;
    if (explicit_ops && (!d || (c[0] & 1) == 0))
        return fail(ctx, PA_EINVAL, d ? "multiplier c must be odd" : "null addend");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    const uint64_t w = words_of(n);
    rc = ensure_staging(ctx, w, explicit_ops);
    if (rc) return rc;
    PA_HIP(ctx, hipMemcpyAsync(ctx->d_key, key, w * 8, hipMemcpyHostToDevice, ctx->stream));
    if (explicit_ops) {
        PA_HIP(ctx, hipMemcpyAsync(ctx->d_c, c, w * 8, hipMemcpyHostToDevice, ctx->stream));
        PA_HIP(ctx, hipMemcpyAsync(ctx->d_d, d, w * 8, hipMemcpyHostToDevice, ctx->stream));
    }
    rc = enqueue(ctx, ctx->d_key, explicit_ops ? ctx->d_c : nullptr,
                 explicit_ops ? ctx->d_d : nullptr, seed_a, seed_b, n, m, ctx->d_out,
                 ctx->stream);
    if (rc) {
        (void)hipStreamSynchronize(ctx->stream);
        return rc;
    }
    PA_HIP(ctx, hipMemcpyAsync(out, ctx->d_out, words_of(m) * 8, hipMemcpyDeviceToHost,
                               ctx->stream));
    PA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PA_OK;
}

int pa_hash(pa_ctx* ctx, const uint64_t* key, uint64_t seed_a, uint64_t seed_b, uint64_t n,
            uint64_t m, uint64_t* out)
{
    return hash_host(ctx, key, nullptr, nullptr, seed_a, seed_b, n, m, out);
}

int pa_hash_ex(pa_ctx* ctx, const uint64_t* key, const uint64_t* c, const uint64_t* d,
               uint64_t n, uint64_t m, uint64_t* out)
{
    if (!c || !d) return ctx ? fail(ctx, PA_EINVAL, "null operand") : PA_EINVAL;
    return hash_host(ctx, key, c, d, 0, 0, n, m, out);
}

struct pa_mul {
    int device;       // where A lives; the creating context may be destroyed first
    uint64_t n;
    uint32_t* A;      // c-hat for blocks of n bits, scaled by 2^32 / L
    Plan plan;        // the geometry c-hat was made with (its spectrum order)
};

int pa_mul_create(pa_ctx* ctx, uint64_t seed_a, const uint64_t* d_c, uint64_t n, void* stream,
                  pa_mul** out)
{
    int rc = check_sizes(ctx, n, 1);
    if (rc) return rc;
    if (!out) return fail(ctx, PA_EINVAL, "null output handle");
    *out = nullptr;
    PA_HIP(ctx, hipSetDevice(ctx->device));
    if (d_c) {
        // read c's low word in the caller's stream order, after whatever wrote it
        uint64_t w0 = 0;
        PA_HIP(ctx, hipMemcpyAsync(&w0, d_c, 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
        PA_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
        if ((w0 & 1) == 0) return fail(ctx, PA_EINVAL, "multiplier c must be odd");
    }
    Plan pl;
    if (!plan_for(ctx, plan_len(n), &pl)) return fail(ctx, PA_EINVAL, "internal: bad pass plan");
    pa_mul* mh = new (std::nothrow) pa_mul;
    if (!mh) return PA_ENOMEM;
    mh->device = ctx->device;
    mh->n = n;
    mh->A = nullptr;
    mh->plan = pl;
    const uint64_t L = pl.L;
    hipError_t e = hipMalloc(&mh->A, (2ull * pl.W + 1) * 4ull * L);
    if (e != hipSuccess) {
        delete mh;
        return fail(ctx, PA_ENOMEM, "multiplier spectrum allocation", e);
    }
    Work w;
    w.c = reinterpret_cast<const uint32_t*>(d_c);
    w.seed_a = seed_a;
    w.n = n;
    w.m = 1;
    w.A = mh->A;
    w.only_chat = true;
    w.key_bytes = (n + 7) / 8;
    w.coeffs = coeffs_of(n, pl.W);
    rc = enqueue_plan(ctx, pl, w, (hipStream_t)stream);
    if (rc) {
        (void)hipFree(mh->A);
        delete mh;
        return rc;
    }
    *out = mh;
    return PA_OK;
}

int pa_hash_mul_async(pa_ctx* ctx, const pa_mul* mh, const uint64_t* d_key, uint64_t seed_b,
                      uint64_t m, uint64_t* d_out, void* stream)
{
    if (!mh) return ctx ? fail(ctx, PA_EINVAL, "null multiplier handle") : PA_EINVAL;
    int rc = check_sizes(ctx, mh->n, m);
    if (rc) return rc;
    if (!d_key || !d_out) return fail(ctx, PA_EINVAL, "null key or output pointer");
    if (mh->device != ctx->device)
        return fail(ctx, PA_EINVAL, "multiplier was made on another device");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    rc = ensure_workspace(ctx, mh->n);
    if (rc) return rc;
    const Plan& pl = mh->plan;
    const uint64_t n = mh->n;
    Work w;
    w.key = reinterpret_cast<const uint32_t*>(d_key);
    w.seed_b = seed_b;
    w.n = n;
    w.m = m;
    w.A = mh->A;
    w.B = ctx->B;
    w.carry = ctx->status;
    w.sums = ctx->A;                   // mh->A holds the cached spectrum
    w.out = d_out;
    w.chunks = chunks_of(digits_of(n), pl.W);
    w.per = carry_digits_per_thread((uint32_t)digits_of(n), pl.W);
    w.key_bytes = (n + 7) / 8;
    w.coeffs = coeffs_of(n, pl.W);
    w.window = window_coeffs(n, m, pl.W);
    w.out_bytes = words_of(m) * 8;
    w.have_chat = true;
    return enqueue_plan(ctx, pl, w, (hipStream_t)stream);
}

void pa_mul_destroy(pa_mul* mh)
{
    if (!mh) return;
    (void)hipSetDevice(mh->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(mh->A);
    delete mh;
}

void pa_batch_destroy(pa_batch* b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_jobs);
    (void)hipFree(b->ws);
    (void)hipFree(b->d_launch);
    (void)hipFree(b->d_ctr);
    if (b->h_abort) (void)hipHostFree(b->h_abort);
    delete b;
}

int pa_batch_create(pa_ctx* ctx, pa_job* jobs, size_t count, pa_batch** out)
{
    return pa_batch_create_ex(ctx, jobs, count, nullptr, out);
}

int pa_batch_create_ex(pa_ctx* ctx, pa_job* jobs, size_t count, const pa_batch_opts* opts,
                       pa_batch** out)
{
    if (!ctx || !out || (!jobs && count)) return PA_EINVAL;
    *out = nullptr;
    const int mode = opts ? opts->mode : PA_BATCH_GROUPED;
    if (mode != PA_BATCH_PERSISTENT && mode != PA_BATCH_GROUPED)
        return fail(ctx, PA_EINVAL, "unknown batch mode");
#if !PA_ENABLE_PERSISTENT
    // The persistent queue kernel hung in its first GPU runs (its queue loop
    // was compiled so that one workgroup repeated one item forever); the
    // corrected loop has not run on a GPU yet, so the mode stays off.
    if (mode == PA_BATCH_PERSISTENT)
        return fail(ctx, PA_EINVAL,
                    "the persistent batch kernel is switched off (not yet validated on a "
                    "GPU); use PA_BATCH_GROUPED");
#endif
    PA_HIP(ctx, hipSetDevice(ctx->device));
    // validate
    std::vector<size_t> ok;
    for (size_t i = 0; i < count; ++i) {
        pa_job& j = jobs[i];
        j.status = PA_OK;
        if (j.n == 0 || j.m == 0 || j.m > j.n || j.n > PA_MAX_N || !j.key || !j.out ||
            (j.c && !j.d) || (!j.c && j.d)) {
            j.status = PA_EINVAL;
            continue;
        }
        if (j.c) {
            uint64_t w0 = 0;
            if (hipMemcpy(&w0, j.c, 8, hipMemcpyDeviceToHost) != hipSuccess) {
                j.status = PA_EDEVICE;
                continue;
            }
            if ((w0 & 1) == 0) {
                j.status = PA_EINVAL;
                continue;
            }
        }
        ok.push_back(i);
    }
    if (ok.empty()) return fail(ctx, PA_EINVAL, "no valid block in the batch");
    std::stable_sort(ok.begin(), ok.end(), [&](size_t a, size_t b) {
        return layout_key(jobs[a].n) < layout_key(jobs[b].n);
    });
    pa_batch* b = new (std::nothrow) pa_batch;
    if (!b) return PA_ENOMEM;
    b->ctx = ctx;
    b->device = ctx->device;
    b->valid = ok.size();
    b->mode = mode;
    // groups and workspace layout
    std::vector<JobDesc> h(ok.size());
    std::vector<uint64_t> offA(ok.size()), offC(ok.size());
    uint64_t bytes = 0;
    for (size_t i = 0; i < ok.size();) {
        const uint64_t key = layout_key(jobs[ok[i]].n);
        size_t e = i;
        uint64_t maxD = 0;
        while (e < ok.size() && layout_key(jobs[ok[e]].n) == key) {
            maxD = std::max<uint64_t>(maxD, digits_of(jobs[ok[e]].n));
            ++e;
        }
        pa_batch::Group g;
        if (!batch_plan(ctx, plan_len(jobs[ok[i]].n), (unsigned)(e - i), &g.plan)) {
            delete b;
            return fail(ctx, PA_EINVAL, "internal: bad pass plan");
        }
        g.first = (uint32_t)i;
        g.count = (uint32_t)(e - i);
        const int W = g.plan.W;
        g.per = mode == PA_BATCH_PERSISTENT ? (W == 3 ? kPersistPer3 : kPersistPer2)
                                            : carry_digits_per_thread((uint32_t)maxD, W);
        const uint64_t chunk = (uint64_t)kCarryThreads * g.per;
        const uint64_t arr = align256((2ull * W + 1) * 4ull * g.plan.L);
        for (size_t k = i; k < e; ++k) {
            const pa_job& j = jobs[ok[k]];
            const uint64_t D = digits_of(j.n);
            JobDesc& d = h[k];
            d.key = reinterpret_cast<const uint32_t*>(j.key);
            d.c = reinterpret_cast<const uint32_t*>(j.c);
            d.d = reinterpret_cast<const uint32_t*>(j.d);
            d.seed_a = j.seed_a;
            d.seed_b = j.seed_b;
            d.n = j.n;
            d.m = j.m;
            d.num_digits = (uint32_t)D;
            d.chunks = (uint32_t)((D + chunk - 1) / chunk);
            d.out = j.out;
            g.chunks = std::max(g.chunks, d.chunks);
            g.key_bytes += (j.n + 7) / 8;
            g.coeffs += coeffs_of(j.n, W);
            g.window += window_coeffs(j.n, j.m, W);
            g.out_bytes += words_of(j.m) * 8;
            offA[k] = bytes;
            bytes += 2 * arr;
            offC[k] = bytes;
            bytes += align256(8ull * d.chunks);
        }
        b->groups.push_back(g);
        i = e;
    }
    b->launches = 0;
    for (const auto& g : b->groups) b->launches += 3 * g.plan.P - 1 + 3;
    if (mode == PA_BATCH_PERSISTENT) b->launches = 2;   // counter reset + the queue kernel
    hipError_t e;
    if ((e = hipMalloc(&b->ws, bytes)) != hipSuccess ||
        (e = hipMalloc(&b->d_jobs, sizeof(JobDesc) * h.size())) != hipSuccess) {
        pa_batch_destroy(b);
        return fail(ctx, PA_ENOMEM, "batch workspace allocation", e);
    }
    b->ws_bytes = bytes;
    for (size_t k = 0; k < h.size(); ++k) {
        h[k].A = reinterpret_cast<uint32_t*>(b->ws + offA[k]);
        h[k].B = reinterpret_cast<uint32_t*>(b->ws + offA[k] + align256(4ull * arr_elems(h[k].n)));
        h[k].carry = reinterpret_cast<uint32_t*>(b->ws + offC[k]);
    }
    if ((e = hipMemcpy(b->d_jobs, h.data(), sizeof(JobDesc) * h.size(), hipMemcpyHostToDevice)) !=
        hipSuccess) {
        pa_batch_destroy(b);
        return fail(ctx, PA_EDEVICE, "batch job table upload", e);
    }
    if (mode == PA_BATCH_PERSISTENT) {
        const int rc = build_persistent(b, opts);
        if (rc) {
            pa_batch_destroy(b);
            return rc;
        }
    }
    *out = b;
    return PA_OK;
}

int pa_batch_run(pa_batch* b, void* stream)
{
    if (!b) return PA_EINVAL;
    pa_ctx* ctx = b->ctx;
    PA_HIP(ctx, hipSetDevice(ctx->device));
    if (b->exec) {
        PA_HIP(ctx, hipGraphLaunch(b->exec, (hipStream_t)stream));
        return PA_OK;
    }
    return enqueue_batch(b, (hipStream_t)stream);
}

int pa_batch_tune(pa_batch* b, int reps)
{
    if (!b) return PA_EINVAL;
    pa_ctx* ctx = b->ctx;
    if (b->mode != PA_BATCH_GROUPED)
        return fail(ctx, PA_EINVAL, "pa_batch_tune: grouped batches only");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    reps = std::max(1, std::min(reps, 100));
    if (!ctx->have_events) {
        for (auto& e : ctx->ev) PA_HIP(ctx, hipEventCreate(&e));
        ctx->have_events = true;
    }
    const hipStream_t st = ctx->stream;
    // a recorded graph holds the old geometries
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    // the clocks rise over tens of milliseconds of load: run the whole batch
    // for about 30 ms first
    for (int i = 0; i < 8; ++i) {
        int rc = enqueue_batch(b, st);
        if (rc) return rc;
    }
    PA_HIP(ctx, hipStreamSynchronize(st));
    for (auto& g : b->groups) {
        const Len len{g.plan.f, g.plan.k};
        Len lw = len;
        lw.W = g.plan.W;
        pa_plan cand[64];
        const int nc = candidates(lw, cand, 64);
        if (nc < 2) continue;
        Work w;
        w.jobs = b->d_jobs + g.first;
        w.batch = g.count;
        w.chunks = g.chunks;
        w.per = g.per;
        // time reps runs of the group alone with geometry pl; two sweeps, the
        // second in reverse order, each candidate keeping its faster time
        auto timed = [&](const Plan& pl, float* ms) -> int {
            PA_HIP(ctx, hipEventRecord(ctx->ev[0], st));
            for (int r = 0; r < reps; ++r) {
                int rc = enqueue_plan(ctx, pl, w, st);
                if (rc) return rc;
            }
            PA_HIP(ctx, hipEventRecord(ctx->ev[1], st));
            PA_HIP(ctx, hipEventSynchronize(ctx->ev[1]));
            PA_HIP(ctx, hipEventElapsedTime(ms, ctx->ev[0], ctx->ev[1]));
            return PA_OK;
        };
        std::vector<Plan> plans(nc);
        std::vector<float> best_ms(nc, 0.f);
        for (int i = 0; i < nc; ++i) {
            const PlanParams pp{cand[i].tile_log,
                                cand[i].strided_tile_log ? cand[i].strided_tile_log : cand[i].tile_log,
                                cand[i].rows3_log};
            if (!make_plan(lw, &plans[i], g.count, pp)) return fail(ctx, PA_EINVAL, "internal: plan");
        }
        for (int sweep = 0; sweep < 2; ++sweep)
            for (int k = 0; k < nc; ++k) {
                const int i = sweep ? nc - 1 - k : k;
                float ms = 0.f;
                int rc = timed(plans[i], &ms);
                if (rc) return rc;
                best_ms[i] = sweep ? std::min(best_ms[i], ms) : ms;
            }
        int bi = 0;
        for (int i = 1; i < nc; ++i)
            if (best_ms[i] < best_ms[bi]) bi = i;
        float cur = 0.f;
        int rc = timed(g.plan, &cur);
        if (rc) return rc;
        if (best_ms[bi] < cur) g.plan = plans[bi];
        g.tuned_ms = std::min(best_ms[bi], cur) / (float)reps;
    }
    return PA_OK;
}

size_t pa_batch_groups(const pa_batch* b) { return b ? b->groups.size() : 0; }

int pa_batch_group(const pa_batch* b, size_t i, uint64_t* length, uint32_t* blocks, pa_plan* plan)
{
    if (!b || i >= b->groups.size()) return PA_EINVAL;
    const auto& g = b->groups[i];
    if (length) *length = g.plan.L;
    if (blocks) *blocks = g.count;
    if (plan) {
        describe(g.plan, plan);
        plan->ms = g.tuned_ms;
    }
    return PA_OK;
}

int pa_batch_capture(pa_batch* b, void* stream)
{
    if (!b) return PA_EINVAL;
    pa_ctx* ctx = b->ctx;
    PA_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    PA_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_batch(b, s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(ctx, PA_EDEVICE, "hipStreamEndCapture", e);
    b->graph = g;
    PA_HIP(ctx, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return PA_OK;
}

uint64_t pa_batch_bytes(const pa_batch* b)
{
    return b ? b->ws_bytes + sizeof(JobDesc) * b->valid + b->table_bytes : 0;
}

size_t pa_batch_size(const pa_batch* b) { return b ? b->valid : 0; }

size_t pa_batch_launches(const pa_batch* b) { return b ? b->launches : 0; }

int pa_hash_many(pa_ctx* ctx, pa_job* jobs, size_t count, void* stream)
{
    pa_batch* b = nullptr;
    int rc = pa_batch_create(ctx, jobs, count, &b);
    if (rc) return rc;
    rc = pa_batch_run(b, stream);
    const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (!rc && e == hipSuccess) rc = pa_batch_result(b);
    pa_batch_destroy(b);
    if (rc) {
        for (size_t i = 0; i < count; ++i)
            if (jobs[i].status == PA_OK) jobs[i].status = rc;
        return rc;
    }
    if (e != hipSuccess) return fail(ctx, PA_EDEVICE, "hipStreamSynchronize", e);
    return PA_OK;
}

int pa_batch_result(const pa_batch* b)
{
    if (!b) return PA_EINVAL;
    if (b->mode == PA_BATCH_PERSISTENT && b->h_abort && *(volatile uint32_t*)b->h_abort)
        return fail(b->ctx, PA_EDEVICE,
                    "persistent batch kernel: a dependency wait gave up; outputs are incomplete");
    return PA_OK;
}

uint64_t pa_toeplitz_length(uint64_t n, uint64_t m, uint64_t* pieces)
{
    ToeplitzPlan tp;
    if (!toeplitz_plan(n, m, &tp)) {
        if (pieces) *pieces = 0;
        return 0;
    }
    if (pieces) *pieces = tp.pieces;
    return tp.len.L();
}

int pa_toeplitz_async(pa_ctx* ctx, const uint64_t* d_key, const uint64_t* d_t, uint64_t seed_t,
                      uint64_t n, uint64_t m, uint64_t* d_out, void* stream)
{
    int rc = check_toeplitz(ctx, n, m);
    if (rc) return rc;
    if (!d_key || !d_out) return fail(ctx, PA_EINVAL, "null key or output pointer");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    const hipStream_t st = (hipStream_t)stream;
    if (!d_t) {
        rc = seeded_t(ctx, seed_t, n + m - 1, st, &d_t);
        if (rc) return rc;
    }
    return enqueue_toeplitz(ctx, d_key, d_t, n, m, d_out, st);
}

int pa_toeplitz(pa_ctx* ctx, const uint64_t* key, const uint64_t* t, uint64_t seed_t, uint64_t n,
                uint64_t m, uint64_t* out)
{
    int rc = check_toeplitz(ctx, n, m);
    if (rc) return rc;
    if (!key || !out) return fail(ctx, PA_EINVAL, "null key or output pointer");
    PA_HIP(ctx, hipSetDevice(ctx->device));
    const uint64_t tw = words_of(n + m - 1);
    rc = ensure_staging(ctx, tw, t != nullptr);
    if (rc) return rc;
    PA_HIP(ctx, hipMemcpyAsync(ctx->d_key, key, words_of(n) * 8, hipMemcpyHostToDevice,
                               ctx->stream));
    const uint64_t* d_t = nullptr;
    if (t) {
        PA_HIP(ctx, hipMemcpyAsync(ctx->d_c, t, tw * 8, hipMemcpyHostToDevice, ctx->stream));
        d_t = ctx->d_c;
    } else {
        rc = seeded_t(ctx, seed_t, n + m - 1, ctx->stream, &d_t);
        if (rc) return rc;
    }
    rc = enqueue_toeplitz(ctx, ctx->d_key, d_t, n, m, ctx->d_out, ctx->stream);
    if (rc) {
        (void)hipStreamSynchronize(ctx->stream);
        return rc;
    }
    PA_HIP(ctx, hipMemcpyAsync(out, ctx->d_out, words_of(m) * 8, hipMemcpyDeviceToHost,
                               ctx->stream));
    PA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PA_OK;
}

int pa_plan_candidates(uint64_t n, pa_plan* out, int max)
{
    if (n == 0 || n > PA_MAX_N || !out || max <= 0) return 0;
    return candidates(plan_len(n), out, max);
}

int pa_plan_get(pa_ctx* ctx, uint64_t n, pa_plan* out)
{
    int rc = check_sizes(ctx, n, 1);
    if (rc) return rc;
    if (!out) return fail(ctx, PA_EINVAL, "null plan");
    Plan pl;
    if (!plan_for(ctx, plan_len(n), &pl)) return fail(ctx, PA_EINVAL, "internal: bad pass plan");
    describe(pl, out);
    return PA_OK;
}

int pa_plan_set(pa_ctx* ctx, uint64_t n, const pa_plan* p)
{
    int rc = check_sizes(ctx, n, 1);
    if (rc) return rc;
    const Len len = plan_len(n);
    const int slot = len_slot(len);
    if (!p) {
        ctx->plans[slot] = pa_ctx::PlanChoice{};
        return PA_OK;
    }
    Plan pl;
    const PlanParams pp{p->tile_log, p->strided_tile_log ? p->strided_tile_log : p->tile_log,
                        len.f == 3 ? p->rows3_log : 0};
    if (pp.t <= 0 || !make_plan(len, &pl, 1, pp))
        return fail(ctx, PA_EINVAL, "plan geometry not valid for this length");
    ctx->plans[slot] = pa_ctx::PlanChoice{pp.t, pp.ts, pp.r0};
    return PA_OK;
}

int pa_tune(pa_ctx* ctx, uint64_t n, int reps, pa_plan* best)
{
    int rc = check_sizes(ctx, n, 1);
    if (rc) return rc;
    PA_HIP(ctx, hipSetDevice(ctx->device));
    reps = std::max(1, std::min(reps, 100));
    rc = ensure_workspace(ctx, n);
    if (rc) return rc;
    if (!ctx->have_events) {
        for (auto& e : ctx->ev) PA_HIP(ctx, hipEventCreate(&e));
        ctx->have_events = true;
    }
    pa_plan cand[64];
    const Len len = plan_len(n);
    const int nc = candidates(len, cand, 64);
    if (nc == 0) return fail(ctx, PA_EINVAL, "internal: no plan");
    const uint64_t m = std::max<uint64_t>(1, n / 2);
    rc = budget_check(ctx, 0, (words_of(n) + words_of(m)) * 8, "tuning buffers");
    if (rc) return rc;
    uint64_t *d_key = nullptr, *d_out = nullptr;
    hipError_t e = hipMalloc(&d_key, words_of(n) * 8);
    if (e == hipSuccess) e = hipMalloc(&d_out, words_of(m) * 8);
    if (e != hipSuccess) {
        (void)hipFree(d_key);
        return fail(ctx, PA_ENOMEM, "tuning buffers", e);
    }
    const hipStream_t st = ctx->stream;
    const int slot = len_slot(len);
    int best_i = 0;
    float best_ms = 0.f;
    rc = PA_OK;
    // Time `count` hashes under the context's current geometry.
    auto timed = [&](int count, float* ms) -> bool {
        if ((e = hipEventRecord(ctx->ev[0], st)) != hipSuccess) return false;
        for (int r = 0; r < count && rc == PA_OK; ++r)
            rc = enqueue(ctx, d_key, nullptr, nullptr, 1, 2, n, m, d_out, st);
        if (rc) return false;
        if ((e = hipEventRecord(ctx->ev[1], st)) != hipSuccess) return false;
        if ((e = hipEventSynchronize(ctx->ev[1])) != hipSuccess) return false;
        return (e = hipEventElapsedTime(ms, ctx->ev[0], ctx->ev[1])) == hipSuccess;
    };
    do {
        if ((e = launch_stream_words(0x243F6A8885A308D3ull, words_of(n), d_key, st)) != hipSuccess)
            break;
        // The clocks rise over tens of milliseconds of sustained load: run the
        // default geometry for about 30 ms before measuring anything.
        ctx->plans[slot] = pa_ctx::PlanChoice{};
        float one = 0.f;
        if (!timed(1, &one)) break;
        const int settle = std::max(2, std::min(500, (int)(30.f / std::max(one, 0.01f))));
        float unused = 0.f;
        if (!timed(settle, &unused)) break;
        // Two sweeps, the second in reverse order; each candidate keeps its
        // faster time, so the order of the list does not bias the choice.
        bool ok = true;
        for (int sweep = 0; sweep < 2 && ok; ++sweep) {
            for (int k = 0; k < nc; ++k) {
                const int i = sweep ? nc - 1 - k : k;
                ctx->plans[slot] = pa_ctx::PlanChoice{cand[i].tile_log,
                                                      cand[i].strided_tile_log ? cand[i].strided_tile_log
                                                                               : cand[i].tile_log,
                                                      cand[i].rows3_log};
                rc = enqueue(ctx, d_key, nullptr, nullptr, 1, 2, n, m, d_out, st);
                float ms = 0.f;
                if (rc || !timed(reps, &ms)) {
                    ok = false;
                    break;
                }
                ms /= reps;
                cand[i].ms = sweep ? std::min(cand[i].ms, ms) : ms;
            }
        }
        if (!ok) break;
        for (int i = 0; i < nc; ++i) {
            if (i == 0 || cand[i].ms < best_ms) {
                best_ms = cand[i].ms;
                best_i = i;
            }
        }
    } while (0);
    (void)hipStreamSynchronize(st);
    (void)hipFree(d_key);
    (void)hipFree(d_out);
    if (rc == PA_OK && e != hipSuccess) rc = fail(ctx, PA_EDEVICE, "pa_tune", e);
    if (rc) {
        ctx->plans[slot] = pa_ctx::PlanChoice{};
        return rc;
    }
    ctx->plans[slot] = pa_ctx::PlanChoice{cand[best_i].tile_log,
                                          cand[best_i].strided_tile_log
                                              ? cand[best_i].strided_tile_log
                                              : cand[best_i].tile_log,
                                          cand[best_i].rows3_log};
    if (best) *best = cand[best_i];
    if (ctx->tune_cache[0]) {
        const auto& pc = ctx->plans[slot];
        if (!append_tuned(ctx->tune_cache, ctx->arch, len, pc.t, pc.ts, pc.r0, best_ms))
            return fail(ctx, PA_EIO, "pa_tune: cannot append to the tuning cache file");
    }
    return PA_OK;
}

}  // extern "C"
