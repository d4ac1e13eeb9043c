// libpa runtime: device context, twiddle tables, plan and workspace, C ABI.
#include <stdio.h>
#include <string.h>

#include <new>

#include "../../include/pa.h"
#include "kernels.h"

using namespace pa;

struct pa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;     // used by the synchronous entry points
    // tables
    uint2* rtw = nullptr;
    uint32_t* pass_lo = nullptr;
    uint32_t* pass_hi = nullptr;
    // workspace, sized for cap_L / cap_D
    uint64_t cap_L = 0, cap_D = 0;
    uint32_t* A = nullptr;            // c-hat   [3][L]
    uint32_t* B = nullptr;            // x-hat, then the product residues [3][L]
    uint32_t* status = nullptr;       // carry state: [chunks] functions, [chunks] carries
    // staging for the synchronous (host memory) entry points
    uint64_t cap_words = 0;
    uint64_t* d_key = nullptr;
    uint64_t* d_c = nullptr;
    uint64_t* d_d = nullptr;
    uint64_t* d_out = nullptr;
    hipEvent_t ev[2 * PA_PROFILE_MAX] = {};
    bool have_events = false;
    char err[512] = {0};
};

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

// Smallest generator of the multiplicative group mod prime p.
uint64_t generator(uint64_t p)
{
    uint64_t f[16];
    int nf = 0;
    uint64_t q = p - 1;
    for (uint64_t d = 2; d * d <= q; ++d) {
        if (q % d == 0) {
            f[nf++] = d;
            while (q % d == 0) q /= d;
        }
    }
    if (q > 1) f[nf++] = q;
    for (uint64_t g = 2; g < p; ++g) {
        bool ok = true;
        for (int i = 0; i < nf && ok; ++i)
            ok = hpow(g, (p - 1) / f[i], p) != 1;
        if (ok) return g;
    }
    return 0;
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

uint64_t words_of(uint64_t bits) { return (bits + 63) / 64; }
uint64_t digits_of(uint64_t bits) { return (bits + 31) / 32; }

int log2_len(uint64_t n)
{
    const uint64_t D = digits_of(n);
    int l = 6;
    while ((1ull << l) < 2 * D - 1) ++l;
    return l;
}

uint32_t chunks_of(uint64_t D)
{
    const uint64_t chunk = (uint64_t)kCarryThreads * carry_digits_per_thread((uint32_t)D);
    return (uint32_t)((D + chunk - 1) / chunk);
}

// Carry state words for the largest chunk count of any block up to D digits.
uint64_t status_words(uint64_t D) { return 2 * ((D + kCarryThreads * 4 - 1) / (kCarryThreads * 4)); }

// Tile size (log2 residues) for a length-2^l transform: whole 2^14 tiles for
// long transforms, smaller ones for short transforms so that there are at
// least 32 tiles per prime to spread over the chip.
#ifndef PA_TILE_SLACK
#define PA_TILE_SLACK 6
#endif

int plan_tile(int l)
{
    if (l <= kTileMinLog) return l;
    int t = l - PA_TILE_SLACK;
    if (t < kTileMinLog) t = kTileMinLog;
    if (t > kTileLog) t = kTileLog;
    return t;
}

// Passes of a length-2^l transform with tiles of 2^t: strided passes of at
// most 2^9 rows (and at least 4 columns per tile), then one contiguous pass
// over whole tiles.
int plan_passes(int l, int t, int* r)
{
    if (l <= t) {
        r[0] = l;
        return 1;
    }
    const int head = l - t;
    const int maxr = (t - 2 < kStridedMaxLog) ? t - 2 : kStridedMaxLog;
    const int k = (head + maxr - 1) / maxr;
    for (int i = 0; i < k; ++i)
        r[i] = head / k + (i < head % k ? 1 : 0);
    r[k] = t;
    return k + 1;
}

// Register steps of a length-2^r in-tile transform in a tile of 2^t residues:
// radix up to 64 in big tiles; smaller radices (more, shorter DFTs per step)
// in small tiles, which have too few threads to hide the latency of long ones.
int plan_steps(int r, int t, int* st)
{
    const int rmax = t >= 13 ? 6 : (t == 12 ? 5 : 4);
    int k = 0;
    while (r > rmax) {
        st[k++] = rmax;
        r -= rmax;
    }
    st[k++] = r;
    return k;
}

void free_workspace(pa_ctx* ctx)
{
    (void)hipFree(ctx->A);
    (void)hipFree(ctx->B);
    (void)hipFree(ctx->status);
    ctx->A = ctx->B = ctx->status = nullptr;
    ctx->cap_L = ctx->cap_D = 0;
}

int ensure_workspace(pa_ctx* ctx, uint64_t n)
{
    const uint64_t L = 1ull << log2_len(n);
    const uint64_t D = digits_of(n);
    if (L <= ctx->cap_L && D <= ctx->cap_D)
        return PA_OK;
    PA_HIP(ctx, hipDeviceSynchronize());
    free_workspace(ctx);
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&ctx->A, kNumPrimes * L * sizeof(uint32_t))) != hipSuccess ||
        (e = hipMalloc(&ctx->B, kNumPrimes * L * sizeof(uint32_t))) != hipSuccess ||
        (e = hipMalloc(&ctx->status, status_words(D) * sizeof(uint32_t))) != hipSuccess) {
        free_workspace(ctx);
        return fail(ctx, PA_ENOMEM, "workspace allocation", e);
    }
    ctx->cap_L = L;
    ctx->cap_D = D;
    return PA_OK;
}

int ensure_staging(pa_ctx* ctx, uint64_t words, bool operands)
{
    if (words <= ctx->cap_words && (!operands || ctx->d_c))
        return PA_OK;
    const uint64_t w = words > ctx->cap_words ? words : ctx->cap_words;
    (void)hipFree(ctx->d_key);
    (void)hipFree(ctx->d_out);
    (void)hipFree(ctx->d_c);
    (void)hipFree(ctx->d_d);
    ctx->d_key = ctx->d_out = ctx->d_c = ctx->d_d = nullptr;
    ctx->cap_words = 0;
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&ctx->d_key, w * 8)) != hipSuccess ||
        (e = hipMalloc(&ctx->d_out, w * 8)) != hipSuccess ||
        (operands && (e = hipMalloc(&ctx->d_c, w * 8)) != hipSuccess) ||
        (operands && (e = hipMalloc(&ctx->d_d, w * 8)) != hipSuccess)) {
        return fail(ctx, PA_ENOMEM, "staging allocation", e);
    }
    ctx->cap_words = w;
    return PA_OK;
}

int check_sizes(pa_ctx* ctx, uint64_t n, uint64_t m)
{
    if (!ctx) return PA_EINVAL;
    if (n == 0 || m == 0 || m > n) return fail(ctx, PA_EINVAL, "need 1 <= m <= n");
    if (n > PA_MAX_N) return fail(ctx, PA_EINVAL, "n exceeds PA_MAX_N");
    return PA_OK;
}

// Optional per-launch event recording for pa_hash_profile.
struct Recorder {
    pa_ctx* ctx;
    pa_profile* prof;
    hipStream_t stream;
    hipError_t begin(int kind, uint64_t bytes)
    {
        const int i = prof->count;
        if (i >= PA_PROFILE_MAX) return hipErrorInvalidValue;
        prof->kind[i] = kind;
        prof->bytes[i] = bytes;
        return hipEventRecord(ctx->ev[2 * i], stream);
    }
    hipError_t end()
    {
        const int i = prof->count++;
        return hipEventRecord(ctx->ev[2 * i + 1], stream);
    }
};

#define PA_LAUNCH(ctx, rec, kind, bytes, call)                                   \
    do {                                                                         \
        if (rec) PA_HIP(ctx, (rec)->begin((kind), (bytes)));                     \
        PA_HIP(ctx, call);                                                       \
        if (rec) PA_HIP(ctx, (rec)->end());                                      \
    } while (0)

// Queue the whole hash on `stream`.  c_digits / d_digits select explicit
// operands (device, 32-bit digit view); null means expand from the seeds.
int enqueue(pa_ctx* ctx, const uint64_t* d_key, const uint64_t* c_words, const uint64_t* d_words,
            uint64_t seed_a, uint64_t seed_b, uint64_t n, uint64_t m, uint64_t* d_out,
            hipStream_t stream, Recorder* rec = nullptr)
{
    int rc = ensure_workspace(ctx, n);
    if (rc) return rc;
    const int l = log2_len(n);
    const uint64_t L = 1ull << l;
    const uint32_t D = (uint32_t)digits_of(n);
    int r[8];
    const int tlog = plan_tile(l);
    const int P = plan_passes(l, tlog, r);
    for (int i = 0; i + 1 < P; ++i)   // strided tiles need >= 4 columns
        if (tlog - r[i] < 2) return fail(ctx, PA_EINVAL, "internal: bad pass plan");
    int s[8];
    {
        int rem = l;
        for (int i = 0; i < P; ++i) {
            rem -= r[i];
            s[i] = rem;
        }
    }
    Tables tb{ctx->pass_lo, ctx->pass_hi};
    const uint64_t arr = kNumPrimes * 4ull * L;        // one residue array
    const uint64_t outD = kNumPrimes * 4ull * D;       // the product coefficients kept

    PassArgs base{};
    base.num_digits = D;
    base.n = n;
    base.logL = l;
    base.logN = tlog;
    base.tb = tb;
    base.rtw = ctx->rtw;
    base.store_limit = (uint32_t)L;
    auto geometry = [&](PassArgs& a, int i) {
        a.r = r[i];
        a.s = s[i];
        a.nsteps = plan_steps(r[i], tlog, a.steps);
    };
    const uint32_t limit = (uint32_t)((D + 3) & ~3ull);   // product digits kept

    // c-hat, scaled on its last pass by 2^32 / L so that the Montgomery
    // pointwise product yields x-hat c-hat / L.
    for (int i = 0; i < P; ++i) {
        PassArgs a = base;
        a.data = ctx->A;
        geometry(a, i);
        a.mode = kForward;
        a.src = kSrcArray;
        if (i == 0) {
            if (c_words) {
                a.src = kSrcDigits;
                a.digits = reinterpret_cast<const uint32_t*>(c_words);
            } else {
                a.src = kSrcSeed;
                a.seed = seed_a;
            }
        }
        if (i == P - 1) {
            a.scale = 1;
            for (int pi = 0; pi < kNumPrimes; ++pi) {
                const uint64_t p = kPrimes[pi];
                const uint64_t w = ((1ull << 32) % p) * hpow(L % p, p - 2, p) % p;
                a.scale_w[pi] = (uint32_t)w;
                a.scale_q[pi] = hshoup(w, p);
            }
        }
        const uint64_t in = (i == 0) ? (c_words ? (n + 7) / 8 : 0) : arr;
        PA_LAUNCH(ctx, rec, PA_K_NTT_PASS, in + arr, launch_pass(a, stream));
    }
    // x-hat, pointwise, and the inverse of the last pass, fused.
    for (int i = 0; i < P; ++i) {
        PassArgs a = base;
        a.data = ctx->B;
        geometry(a, i);
        a.mode = (i == P - 1) ? kFused : kForward;
        if (P == 1) a.store_limit = limit;
        a.other = ctx->A;
        a.src = (i == 0) ? kSrcDigits : kSrcArray;
        a.digits = reinterpret_cast<const uint32_t*>(d_key);
        uint64_t in = (i == 0) ? (n + 7) / 8 : arr, outb = arr;
        if (i == P - 1) {
            in += arr;                       // c-hat
            if (P == 1) outb = outD;         // also the last inverse pass
        }
        const uint64_t bytes = in + outb;
        PA_LAUNCH(ctx, rec, PA_K_NTT_PASS, bytes, launch_pass(a, stream));
    }
    // remaining inverse passes
    for (int i = P - 2; i >= 0; --i) {
        PassArgs a = base;
        a.data = ctx->B;
        geometry(a, i);
        a.mode = kInverse;
        a.src = kSrcArray;
        if (i == 0) a.store_limit = limit;
        PA_LAUNCH(ctx, rec, PA_K_NTT_PASS, arr + (i == 0 ? outD : arr), launch_pass(a, stream));
    }
    CarryArgs ca{};
    ca.res = ctx->B;
    ca.L = (uint32_t)L;
    ca.num_digits = D;
    ca.n = n;
    ca.m = m;
    if (d_words) {
        ca.addend_src = kSrcDigits;
        ca.addend = reinterpret_cast<const uint32_t*>(d_words);
    } else {
        ca.addend_src = kSrcSeed;
        ca.seed = seed_b;
    }
    ca.chunks = chunks_of(D);
    ca.desc = ctx->status;
    ca.carry_in = ctx->status + ca.chunks;
    ca.out = d_out;
    PA_LAUNCH(ctx, rec, PA_K_CARRY_LOCAL, outD + 4ull * ca.chunks, launch_carry_local(ca, stream));
    PA_LAUNCH(ctx, rec, PA_K_CARRY_SCAN, 8ull * ca.chunks, launch_carry_scan(ca, stream));
    PA_LAUNCH(ctx, rec, PA_K_CARRY_APPLY, outD + 4ull * ca.chunks + words_of(m) * 8,
              launch_carry_apply(ca, stream));
    return PA_OK;
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
    default: return "unknown status";
    }
}

const char* pa_last_error(const pa_ctx* ctx) { return ctx ? ctx->err : ""; }

uint64_t pa_transform_length(uint64_t n)
{
    if (n == 0 || n > PA_MAX_N) return 0;
    return 1ull << log2_len(n);
}

uint64_t pa_workspace_bytes(uint64_t n)
{
    if (n == 0 || n > PA_MAX_N) return 0;
    const uint64_t L = 1ull << log2_len(n);
    const uint64_t D = digits_of(n);
    return 2 * kNumPrimes * L * 4 + status_words(D) * 4;
}

int pa_init(pa_ctx** out, int device)
{
    if (!out) return PA_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return PA_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PA_ENODEV;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PA_ENODEV;

    pa_ctx* ctx = new (std::nothrow) pa_ctx;
    if (!ctx) return PA_ENOMEM;
    ctx->device = device;
    int rc = PA_OK;
    uint2* h_tile = nullptr;
    uint32_t *h_lo = nullptr, *h_hi = nullptr;
    do {
        if (hipSetDevice(device) != hipSuccess) { rc = PA_ENODEV; break; }
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            rc = PA_EDEVICE;
            break;
        }
        h_tile = new (std::nothrow) uint2[kNumPrimes * 64];
        h_lo = new (std::nothrow) uint32_t[kNumPrimes * 4096];
        h_hi = new (std::nothrow) uint32_t[kNumPrimes * 8192];
        if (!h_tile || !h_lo || !h_hi) { rc = PA_ENOMEM; break; }
        for (int pi = 0; pi < kNumPrimes; ++pi) {
            const uint64_t p = kPrimes[pi];
            const uint64_t g = generator(p);
            const uint64_t w25 = hpow(g, (p - 1) >> kLogMaxLen, p);   // order 2^25
            const uint64_t w6 = hpow(w25, 1ull << (kLogMaxLen - 6), p);     // order 64
            const uint64_t w6i = hpow(w6, p - 2, p);
            for (int e = 0; e < 32; ++e) {
                const uint64_t f = hpow(w6, e, p), b = hpow(w6i, e, p);
                h_tile[pi * 64 + e] = make_uint2((uint32_t)f, hshoup(f, p));
                h_tile[pi * 64 + 32 + e] = make_uint2((uint32_t)b, hshoup(b, p));
            }
            uint64_t w = 1;
            for (int i = 0; i < 4096; ++i) {
                h_lo[pi * 4096 + i] = hmont(w, p);
                w = w * w25 % p;
            }
            const uint64_t step = hpow(w25, 4096, p);
            w = 1;
            for (int j = 0; j < 8192; ++j) {
                h_hi[pi * 8192 + j] = hmont(w, p);
                w = w * step % p;
            }
        }
        if (hipMalloc(&ctx->rtw, sizeof(uint2) * kNumPrimes * 64) != hipSuccess ||
            hipMalloc(&ctx->pass_lo, sizeof(uint32_t) * kNumPrimes * 4096) != hipSuccess ||
            hipMalloc(&ctx->pass_hi, sizeof(uint32_t) * kNumPrimes * 8192) != hipSuccess) {
            rc = PA_ENOMEM;
            break;
        }
        if (hipMemcpy(ctx->rtw, h_tile, sizeof(uint2) * kNumPrimes * 64,
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->pass_lo, h_lo, sizeof(uint32_t) * kNumPrimes * 4096,
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->pass_hi, h_hi, sizeof(uint32_t) * kNumPrimes * 8192,
                      hipMemcpyHostToDevice) != hipSuccess) {
            rc = PA_EDEVICE;
            break;
        }
    } while (0);
    delete[] h_tile;
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
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_workspace(ctx);
    (void)hipFree(ctx->d_key);
    (void)hipFree(ctx->d_out);
    (void)hipFree(ctx->d_c);
    (void)hipFree(ctx->d_d);
    (void)hipFree(ctx->rtw);
    (void)hipFree(ctx->pass_lo);
    (void)hipFree(ctx->pass_hi);
    if (ctx->have_events)
        for (auto& e : ctx->ev) (void)hipEventDestroy(e);
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

}  // extern "C"
