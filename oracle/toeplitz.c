/*
 * CPU oracle for the Toeplitz-hash variant.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests and the benchmark's checks do.  It shares no
 * code, header, table or constant with the GPU path.
 *
 * The paper names the Toeplitz family as the usual privacy-amplification hash
 * and the foil of its modular-arithmetic family (Introduction) without writing
 * it out.  The standard member (Krawczyk, CRYPTO 1994; Mansour, Nisan and
 * Tiwari, STOC 1990) is an m x n matrix over GF(2) that is constant along its
 * diagonals, fixed by n + m - 1 random bits t_0 .. t_{n+m-2}:
 *
 *     T[i][j] = t[i - j + n - 1],      y = T x over GF(2),
 *     y_i = XOR_{j < n} ( t[i + n - 1 - j] AND x_j ),   0 <= i < m.
 *
 * Bits are packed as for the modular hash: bit i of a value is bit i%64 of
 * 64-bit word i/64; bits past the stated length in the top word are ignored on
 * input and written as zero on output.  A seeded t is the stream of seed_t
 * (SplitMix64 in counter form, as in pa_oracle.c) masked to n + m - 1 bits.
 *
 * Evaluation is the definition itself: with x reversed (xr_k = x_{n-1-k}),
 * y_i = parity( popcount( bits [i, i+n) of t  AND  xr ) ), one window per
 * output bit; output bits are split into ranges over POSIX threads.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

uint64_t oracle_splitmix64(uint64_t seed, uint64_t i);
void oracle_expand_operand(uint64_t seed, uint64_t n, int force_odd, uint64_t *out);

static size_t nwords(uint64_t bits) { return (size_t)((bits + 63) / 64); }

static int bit_of(const uint64_t *v, uint64_t i) { return (int)((v[i / 64] >> (i % 64)) & 1u); }

/* x reversed over n bits: bit k of the result is bit n-1-k of x. */
static uint64_t *reversed(const uint64_t *x, uint64_t n)
{
    uint64_t *r = calloc(nwords(n) + 1, sizeof(uint64_t));
    if (!r)
        return NULL;
    for (uint64_t k = 0; k < n; k++)
        if (bit_of(x, n - 1 - k))
            r[k / 64] |= 1ull << (k % 64);
    return r;
}

/* y_i for one i: parity of (bits [i, i+n) of t) AND xr. */
static int output_bit(const uint64_t *t, const uint64_t *xr, uint64_t n, uint64_t i)
{
    const size_t w = nwords(n);
    const size_t base = (size_t)(i / 64);
    const unsigned s = (unsigned)(i % 64);
    uint64_t acc = 0;
    for (size_t k = 0; k < w; k++) {
        uint64_t win = t[base + k] >> s;
        if (s)
            win |= t[base + k + 1] << (64 - s);
        acc ^= win & xr[k];
    }
    return __builtin_popcountll(acc) & 1;
}

struct range_job {
    const uint64_t *t, *xr;
    uint64_t n, lo, hi;
    uint64_t *out;           /* words lo/64 .. (hi-1)/64, lo a multiple of 64 */
};

static void *range_run(void *p)
{
    struct range_job *j = p;
    for (uint64_t i = j->lo; i < j->hi; i++)
        if (output_bit(j->t, j->xr, j->n, i))
            j->out[i / 64] |= 1ull << (i % 64);
    return NULL;
}

/* t padded with one zero word (the window of the last output reads one word past). */
static uint64_t *padded_t(const uint64_t *t, uint64_t bits)
{
    const size_t w = nwords(bits);
    uint64_t *p = calloc(w + 1, sizeof(uint64_t));
    if (!p)
        return NULL;
    memcpy(p, t, w * sizeof(uint64_t));
    if (bits % 64)
        p[w - 1] &= (1ull << (bits % 64)) - 1;
    return p;
}

/*
 * y = T x for explicit t (n + m - 1 bits).  out: nwords(m) words.  threads:
 * worker threads (<= 1: the calling thread).  Returns 0, or -1 for invalid
 * sizes or allocation failure.
 */
int oracle_toeplitz_ex(const uint64_t *key, const uint64_t *t, uint64_t n, uint64_t m,
                       uint64_t *out, int threads)
{
    if (n == 0 || m == 0 || !key || !t || !out)
        return -1;
    uint64_t *x = calloc(nwords(n), sizeof(uint64_t));
    if (!x)
        return -1;
    memcpy(x, key, nwords(n) * sizeof(uint64_t));
    if (n % 64)
        x[nwords(n) - 1] &= (1ull << (n % 64)) - 1;
    uint64_t *xr = reversed(x, n);
    uint64_t *tp = padded_t(t, n + m - 1);
    free(x);
    if (!xr || !tp) {
        free(xr); free(tp);
        return -1;
    }
    memset(out, 0, nwords(m) * sizeof(uint64_t));
    if (threads < 1)
        threads = 1;
    if (threads > 64)
        threads = 64;
    /* ranges on 64-bit boundaries so that no two threads write one word */
    const uint64_t mw = nwords(m);
    const uint64_t per = (mw + threads - 1) / threads;
    pthread_t th[64];
    struct range_job jobs[64];
    int started = 0;
    for (int k = 0; k < threads; k++) {
        uint64_t lo = (uint64_t)k * per * 64, hi = lo + per * 64;
        if (hi > m) hi = m;
        if (lo >= hi) break;
        jobs[k] = (struct range_job){tp, xr, n, lo, hi, out};
        if (threads > 1 && pthread_create(&th[k], NULL, range_run, &jobs[k]) == 0) {
            started = k + 1;
        } else {
            range_run(&jobs[k]);
        }
    }
    for (int k = 0; k < started; k++)
        pthread_join(th[k], NULL);
    free(xr);
    free(tp);
    return 0;
}

/* Same with t drawn from seed_t (n + m - 1 bits). */
int oracle_toeplitz(const uint64_t *key, uint64_t seed_t, uint64_t n, uint64_t m, uint64_t *out,
                    int threads)
{
    if (n == 0 || m == 0)
        return -1;
    uint64_t *t = calloc(nwords(n + m - 1), sizeof(uint64_t));
    if (!t)
        return -1;
    oracle_expand_operand(seed_t, n + m - 1, 0, t);
    int rc = oracle_toeplitz_ex(key, t, n, m, out, threads);
    free(t);
    return rc;
}

/*
 * Selected output bits only: bits[k] = y_{idx[k]} (each idx[k] < m), for
 * checking large blocks at sampled positions.  Returns 0 or -1.
 */
int oracle_toeplitz_bits(const uint64_t *key, const uint64_t *t, uint64_t n, uint64_t m,
                         const uint64_t *idx, uint64_t count, uint8_t *bits)
{
    if (n == 0 || m == 0 || !key || !t || (count && (!idx || !bits)))
        return -1;
    uint64_t *x = calloc(nwords(n), sizeof(uint64_t));
    if (!x)
        return -1;
    memcpy(x, key, nwords(n) * sizeof(uint64_t));
    if (n % 64)
        x[nwords(n) - 1] &= (1ull << (n % 64)) - 1;
    uint64_t *xr = reversed(x, n);
    uint64_t *tp = padded_t(t, n + m - 1);
    free(x);
    if (!xr || !tp) {
        free(xr); free(tp);
        return -1;
    }
    int rc = 0;
    for (uint64_t k = 0; k < count; k++) {
        if (idx[k] >= m) { rc = -1; break; }
        bits[k] = (uint8_t)output_bit(tp, xr, n, idx[k]);
    }
    free(xr);
    free(tp);
    return rc;
}

/*
 * For x != y (n-bit), the number of the 2^(n+m-1) matrices T with T x = T y,
 * every member evaluated with oracle_toeplitz_ex; n + m - 1 <= 22.
 */
int64_t oracle_toeplitz_collision_count(uint64_t n, uint64_t m, uint64_t x, uint64_t y)
{
    if (n == 0 || m == 0 || n > 20 || n + m - 1 > 22)
        return -1;
    const uint64_t mask = (1ull << n) - 1;
    x &= mask;
    y &= mask;
    int64_t count = 0;
    for (uint64_t t = 0; t < (1ull << (n + m - 1)); t++) {
        uint64_t gx = 0, gy = 0;
        oracle_toeplitz_ex(&x, &t, n, m, &gx, 1);
        oracle_toeplitz_ex(&y, &t, n, m, &gy, 1);
        count += (gx == gy);
    }
    return count;
}
