/*
 * CPU oracle for the G_{c,d} privacy-amplification hash.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant with the GPU path.
 *
 * What it computes (Section 2.3, eq. (6) and the g_{c,d} definition after it,
 * with the pipeline of Section 3.2: multiply-add, reduce mod 2^n, export, keep
 * the most significant r bits):
 *
 *     V = (c * x + d) mod 2^n,      y = floor(V / 2^(n - m))   (m output bits)
 *
 * x, c, d are n-bit integers held as little-endian arrays of 64-bit limbs
 * (limb 0 least significant, bit i of a value is bit i%64 of limb i/64).  Bits
 * at positions >= n in the top limb of an input are ignored.  The output y is
 * ceil(m/64) limbs in the same order with bits >= m of the top limb zero.
 *
 * The product c*x mod 2^n is a low-half product: schoolbook for short operands,
 * Karatsuba above a threshold.  Both are written out plainly; no FFT, no
 * library big-integer code.  For operands of many limbs the three Karatsuba
 * sub-products of the top levels run on separate POSIX threads.
 *
 * Seed expansion (the paper only says g is chosen at random, Section 2.2): word
 * i of the stream for seed s is the i-th output of SplitMix64 seeded with s
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014), i.e. mix(s + (i+1) * 0x9E3779B97F4A7C15).  c is the stream of
 * seed_a masked to n bits with bit 0 forced to 1 (eq. (6) requires c odd); d is
 * the stream of seed_b masked to n bits.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t limb;
typedef unsigned __int128 dlimb;

#define SCHOOL_LIMBS 32          /* schoolbook at or below this many limbs */
#define PAR_MIN_LIMBS 4096       /* split onto threads only above this size */

/* ------------------------------------------------------------------------ */
/* SplitMix64, counter form                                                  */
/* ------------------------------------------------------------------------ */

uint64_t oracle_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static size_t words_of(uint64_t bits) { return (size_t)((bits + 63) / 64); }

/* Clear the bits at positions >= n of an array of words_of(n) limbs. */
static void mask_bits(limb *v, uint64_t n)
{
    size_t w = words_of(n);
    unsigned r = (unsigned)(n % 64);
    if (r)
        v[w - 1] &= (((limb)1) << r) - 1;
}

/* Operand of n bits drawn from seed; force_odd sets bit 0 (the multiplier c). */
void oracle_expand_operand(uint64_t seed, uint64_t n, int force_odd, uint64_t *out)
{
    size_t w = words_of(n);
    for (size_t i = 0; i < w; i++)
        out[i] = oracle_splitmix64(seed, i);
    mask_bits(out, n);
    if (force_odd)
        out[0] |= 1;
}

/* ------------------------------------------------------------------------ */
/* Limb-array helpers                                                        */
/* ------------------------------------------------------------------------ */

/* r[0..n) += a[0..n); returns the carry out of limb n-1. */
static limb add_n(limb *r, const limb *a, size_t n)
{
    limb carry = 0;
    for (size_t i = 0; i < n; i++) {
        dlimb t = (dlimb)r[i] + a[i] + carry;
        r[i] = (limb)t;
        carry = (limb)(t >> 64);
    }
    return carry;
}

/* r[0..rn) += a[0..an), an <= rn; returns the carry out of limb rn-1. */
static limb add_into(limb *r, size_t rn, const limb *a, size_t an)
{
    limb carry = add_n(r, a, an);
    for (size_t i = an; i < rn && carry; i++) {
        r[i] += 1;
        carry = (r[i] == 0);
    }
    return carry;
}

/* r[0..rn) -= a[0..an), an <= rn; returns the borrow out of limb rn-1. */
static limb sub_into(limb *r, size_t rn, const limb *a, size_t an)
{
    limb borrow = 0;
    for (size_t i = 0; i < an; i++) {
        limb ri = r[i], ai = a[i];
        limb d = ri - ai - borrow;
        borrow = (ri < ai) || (ri == ai && borrow);
        r[i] = d;
    }
    for (size_t i = an; i < rn && borrow; i++) {
        borrow = (r[i] == 0);
        r[i] -= 1;
    }
    return borrow;
}

/* ------------------------------------------------------------------------ */
/* Full product r[0..2n) = a[0..n) * b[0..n)                                 */
/* ------------------------------------------------------------------------ */

static void mul_school(limb *r, const limb *a, const limb *b, size_t n)
{
    memset(r, 0, 2 * n * sizeof(limb));
    for (size_t i = 0; i < n; i++) {
        limb carry = 0;
        for (size_t j = 0; j < n; j++) {
            dlimb t = (dlimb)a[i] * b[j] + r[i + j] + carry;
            r[i + j] = (limb)t;
            carry = (limb)(t >> 64);
        }
        r[i + n] = carry;
    }
}

static void mul_full(limb *r, const limb *a, const limb *b, size_t n, int par);

struct mul_job {
    limb *r;
    const limb *a, *b;
    size_t n;
    int par;
};

static void *mul_job_run(void *p)
{
    struct mul_job *j = (struct mul_job *)p;
    mul_full(j->r, j->a, j->b, j->n, j->par);
    return NULL;
}

/*
 * Karatsuba: with l = ceil(n/2), h = n - l, a = a0 + a1 B^l, b = b0 + b1 B^l,
 *   a b = z0 + B^l (z1 - z0 - z2) + B^(2l) z2,
 *   z0 = a0 b0, z2 = a1 b1, z1 = (a0 + a1)(b0 + b1).
 * a0 + a1 may carry one bit beyond l limbs; the product of the two sums is then
 * taken over l+1 limbs so nothing is dropped.  `par` levels of the recursion
 * compute their three sub-products on separate threads.
 */
static void mul_full(limb *r, const limb *a, const limb *b, size_t n, int par)
{
    if (n <= SCHOOL_LIMBS) {
        mul_school(r, a, b, n);
        return;
    }
    size_t l = (n + 1) / 2, h = n - l, s = l + 1;
    limb *sa = calloc(s, sizeof(limb));
    limb *sb = calloc(s, sizeof(limb));
    limb *z1 = calloc(2 * s, sizeof(limb));
    limb *z0 = r;              /* 2l limbs  */
    limb *z2 = calloc(2 * h > 0 ? 2 * h : 1, sizeof(limb));

    memcpy(sa, a, l * sizeof(limb));
    sa[l] = add_into(sa, l, a + l, h);
    memcpy(sb, b, l * sizeof(limb));
    sb[l] = add_into(sb, l, b + l, h);

    if (par > 0 && n >= PAR_MIN_LIMBS) {
        struct mul_job jobs[3] = {
            { z0, a, b, l, par - 1 },
            { z2, a + l, b + l, h, par - 1 },
            { z1, sa, sb, s, par - 1 },
        };
        pthread_t t[2];
        int started[2] = { 0, 0 };
        for (int i = 0; i < 2; i++)
            started[i] = pthread_create(&t[i], NULL, mul_job_run, &jobs[i]) == 0;
        mul_job_run(&jobs[2]);
        for (int i = 0; i < 2; i++) {
            if (started[i])
                pthread_join(t[i], NULL);
            else
                mul_job_run(&jobs[i]);
        }
    } else {
        mul_full(z0, a, b, l, 0);
        mul_full(z2, a + l, b + l, h, 0);
        mul_full(z1, sa, sb, s, 0);
    }

    /* z1 <- z1 - z0 - z2 (non-negative; fits in 2s limbs) */
    sub_into(z1, 2 * s, z0, 2 * l);
    sub_into(z1, 2 * s, z2, 2 * h);

    /* r = z0 (already in r[0..2l)) + z2 B^(2l) + z1 B^l */
    memcpy(r + 2 * l, z2, 2 * h * sizeof(limb));
    /* z1 < 2^(64 (2l + 1)); its top limbs beyond what fits are zero */
    size_t z1n = 2 * s;
    while (z1n > 0 && z1[z1n - 1] == 0)
        z1n--;
    if (z1n > 2 * n - l)
        z1n = 2 * n - l;  /* the true value fits; higher limbs are zero */
    add_into(r + l, 2 * n - l, z1, z1n);

    free(sa);
    free(sb);
    free(z1);
    free(z2);
}

/* ------------------------------------------------------------------------ */
/* Low-half product r[0..n) = (a[0..n) * b[0..n)) mod B^n                    */
/* ------------------------------------------------------------------------ */

static void mul_low_school(limb *r, const limb *a, const limb *b, size_t n)
{
    memset(r, 0, n * sizeof(limb));
    for (size_t i = 0; i < n; i++) {
        limb carry = 0;
        for (size_t j = 0; i + j < n; j++) {
            dlimb t = (dlimb)a[i] * b[j] + r[i + j] + carry;
            r[i + j] = (limb)t;
            carry = (limb)(t >> 64);
        }
    }
}

static void mul_low(limb *r, const limb *a, const limb *b, size_t n, int par);

struct low_job {
    limb *r;
    const limb *a, *b;
    size_t n;
    int par;
    int full;
};

static void *low_job_run(void *p)
{
    struct low_job *j = (struct low_job *)p;
    if (j->full)
        mul_full(j->r, j->a, j->b, j->n, j->par);
    else
        mul_low(j->r, j->a, j->b, j->n, j->par);
    return NULL;
}

/*
 * With l = ceil(n/2), h = n - l (h <= l):
 *   (a b) mod B^n = [a0 b0 + B^l (a0 b1 + a1 b0)] mod B^n,
 * and modulo B^n the two cross terms only need their low h limbs, which depend
 * only on the low h limbs of a0 and b0:  lo_h(a0[0..h) b1) + lo_h(a1 b0[0..h)).
 * The a1 b1 B^(2l) term is a multiple of B^n and drops out.
 */
static void mul_low(limb *r, const limb *a, const limb *b, size_t n, int par)
{
    if (n <= SCHOOL_LIMBS) {
        mul_low_school(r, a, b, n);
        return;
    }
    size_t l = (n + 1) / 2, h = n - l;
    limb *z0 = malloc(2 * l * sizeof(limb));
    limb *t1 = malloc(h * sizeof(limb));
    limb *t2 = malloc(h * sizeof(limb));

    if (par > 0 && n >= PAR_MIN_LIMBS) {
        struct low_job jobs[3] = {
            { t1, a, b + l, h, par - 1, 0 },
            { t2, a + l, b, h, par - 1, 0 },
            { z0, a, b, l, par - 1, 1 },
        };
        pthread_t t[2];
        int started[2] = { 0, 0 };
        for (int i = 0; i < 2; i++)
            started[i] = pthread_create(&t[i], NULL, low_job_run, &jobs[i]) == 0;
        low_job_run(&jobs[2]);
        for (int i = 0; i < 2; i++) {
            if (started[i])
                pthread_join(t[i], NULL);
            else
                low_job_run(&jobs[i]);
        }
    } else {
        mul_full(z0, a, b, l, 0);
        mul_low(t1, a, b + l, h, 0);
        mul_low(t2, a + l, b, h, 0);
    }

    memcpy(r, z0, n * sizeof(limb));
    add_n(r + l, t1, h);   /* carries out of limb n-1 are discarded (mod B^n) */
    add_n(r + l, t2, h);

    free(z0);
    free(t1);
    free(t2);
}

/* ------------------------------------------------------------------------ */
/* The hash                                                                  */
/* ------------------------------------------------------------------------ */

/* Bits [lo, lo + m) of v (words_of(n) limbs) into out (words_of(m) limbs). */
static void extract_bits(const limb *v, uint64_t lo, uint64_t m, limb *out)
{
    size_t ow = words_of(m);
    size_t base = (size_t)(lo / 64);
    unsigned sh = (unsigned)(lo % 64);
    size_t vw = words_of(lo + m);
    for (size_t i = 0; i < ow; i++) {
        limb w = v[base + i] >> sh;
        if (sh && base + i + 1 < vw)
            w |= v[base + i + 1] << (64 - sh);
        out[i] = w;
    }
    mask_bits(out, m);
}

/*
 * y = floor(((c x + d) mod 2^n) / 2^(n-m)).  key, c, d: words_of(n) limbs
 * (bits >= n ignored); out: words_of(m) limbs.  par_levels: number of top
 * Karatsuba levels whose three sub-products run on threads (0 = single
 * thread; level k uses up to 3^k threads).  Returns 0, or -1 for invalid sizes or allocation failure.
 */
int oracle_pa_hash_ex(const uint64_t *key, const uint64_t *c, const uint64_t *d,
                      uint64_t n, uint64_t m, uint64_t *out, int par_levels)
{
    if (n == 0 || m == 0 || m > n || !key || !c || !d || !out)
        return -1;
    size_t w = words_of(n);
    limb *x = malloc(w * sizeof(limb));
    limb *cc = malloc(w * sizeof(limb));
    limb *dd = malloc(w * sizeof(limb));
    limb *v = malloc(w * sizeof(limb));
    if (!x || !cc || !dd || !v) {
        free(x); free(cc); free(dd); free(v);
        return -1;
    }
    memcpy(x, key, w * sizeof(limb));
    memcpy(cc, c, w * sizeof(limb));
    memcpy(dd, d, w * sizeof(limb));
    mask_bits(x, n);
    mask_bits(cc, n);
    mask_bits(dd, n);

    mul_low(v, cc, x, w, par_levels);   /* (c x) mod 2^(64 w)         */
    add_n(v, dd, w);                    /* + d, mod 2^(64 w)          */
    mask_bits(v, n);                    /* mod 2^n                    */
    extract_bits(v, n - m, m, out);     /* the most significant m bits */

    free(x); free(cc); free(dd); free(v);
    return 0;
}

/* Same with c and d expanded from seeds (c forced odd). */
int oracle_pa_hash(const uint64_t *key, uint64_t seed_a, uint64_t seed_b,
                   uint64_t n, uint64_t m, uint64_t *out, int par_levels)
{
    if (n == 0 || m == 0 || m > n || !key || !out)
        return -1;
    size_t w = words_of(n);
    limb *c = malloc(w * sizeof(limb));
    limb *d = malloc(w * sizeof(limb));
    if (!c || !d) {
        free(c); free(d);
        return -1;
    }
    oracle_expand_operand(seed_a, n, 1, c);
    oracle_expand_operand(seed_b, n, 0, d);
    int rc = oracle_pa_hash_ex(key, c, d, n, m, out, par_levels);
    free(c);
    free(d);
    return rc;
}

/* Full product exposed for self-tests: r[0..2n) = a[0..n) b[0..n). */
void oracle_mul_full(const uint64_t *a, const uint64_t *b, uint64_t n, uint64_t *r)
{
    mul_full(r, a, b, (size_t)n, 0);
}

/* Low product exposed for self-tests: r[0..n) = a b mod B^n. */
void oracle_mul_low(const uint64_t *a, const uint64_t *b, uint64_t n, uint64_t *r, int par)
{
    mul_low(r, a, b, (size_t)n, par);
}

/*
 * delta_G(x, y) of eq. (4) for the whole family G_{c,d} of eq. (6) at input
 * size n <= 20: the number of (c odd, d) in Z_{2^n} with g(x) = g(y), x != y.
 * Every member is evaluated with the hash above.  Returns -1 on bad arguments.
 */
int64_t oracle_collision_count(uint64_t n, uint64_t m, uint64_t x, uint64_t y)
{
    if (n == 0 || n > 20 || m == 0 || m > n)
        return -1;
    uint64_t mask = (((uint64_t)1) << n) - 1;
    x &= mask;
    y &= mask;
    if (x == y)
        return 0;   /* delta is 0 for x == y by eq. (3) */
    int64_t count = 0;
    for (uint64_t c = 1; c <= mask; c += 2) {
        for (uint64_t d = 0; d <= mask; d++) {
            uint64_t gx, gy;
            oracle_pa_hash_ex(&x, &c, &d, n, m, &gx, 0);
            oracle_pa_hash_ex(&y, &c, &d, n, m, &gy, 0);
            count += (gx == gy);
        }
    }
    return count;
}
