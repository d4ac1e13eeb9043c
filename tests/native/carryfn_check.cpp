// Host check of the carry-transfer functions in carryfn.h: every position's
// function against (s + c) >> 32, composition against function application
// for every pair and triple of valid functions, and long random carry chains
// (with column sums near 2^32 boundaries) against sequential propagation.
#include <stdio.h>
#include <stdint.h>

#include <random>
#include <vector>

#include "carryfn.h"

using namespace pa;

static int fails = 0;
#define CHECK(cond)                                                           \
    do {                                                                      \
        if (!(cond)) {                                                        \
            if (fails++ < 10) fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #cond); \
        }                                                                     \
    } while (0)

// The map {0..3} -> {0..3} of a function code, as four values.
static void table(uint32_t f, uint32_t out[4])
{
    for (uint32_t c = 0; c < 4; ++c) out[c] = carry_apply(f, c);
}

int main()
{
    // 1. one position: f(c) = (s + c) >> 32 for every column sum that occurs
    //    (s <= 4 * 2^32 - 4, so that carries stay in 0..3)
    std::vector<uint64_t> sums;
    const uint32_t los[] = {0u, 1u, 2u, 3u, 4u, 5u, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFF8u,
                            0xFFFFFFF9u, 0xFFFFFFFAu, 0xFFFFFFFBu, 0xFFFFFFFCu, 0xFFFFFFFDu,
                            0xFFFFFFFEu, 0xFFFFFFFFu};
    for (uint64_t hi = 0; hi < 4; ++hi)
        for (uint32_t lo : los)
            if (hi * (1ull << 32) + lo <= 4 * (1ull << 32) - 4) sums.push_back(hi * (1ull << 32) + lo);
    for (uint64_t s : sums)
        for (uint32_t c = 0; c < 4; ++c)
            CHECK(carry_apply(carry_fn_of_sum(s), c) == (uint32_t)((s + c) >> 32));

    // 2. all functions that runs of positions can have: the position functions
    //    and everything composed from them (closure), plus the identity
    std::vector<uint32_t> fs;
    for (uint64_t s : sums) {
        const uint32_t f = carry_fn_of_sum(s);
        bool seen = false;
        for (uint32_t g : fs) seen |= g == f;
        if (!seen) fs.push_back(f);
    }
    for (size_t grow = 1; grow;) {
        grow = 0;
        const size_t n = fs.size();
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j < n; ++j) {
                const uint32_t h = carry_compose(fs[i], fs[j]);
                bool seen = false;
                for (uint32_t g : fs) seen |= g == h;
                if (!seen) { fs.push_back(h); ++grow; }
            }
    }
    fs.push_back(kCarryIdentity);
    for (uint32_t f : fs)
        for (uint32_t g : fs) {
            uint32_t tf[4], tg[4], th[4];
            table(f, tf);
            table(g, tg);
            table(carry_compose(f, g), th);
            for (int c = 0; c < 4; ++c) {
                CHECK(tf[c] < 4 && tg[c] < 4);
                CHECK(th[c] == tg[tf[c]]);
            }
            for (uint32_t h : fs) {
                uint32_t a[4], b[4];
                table(carry_compose(carry_compose(f, g), h), a);
                table(carry_compose(f, carry_compose(g, h)), b);
                for (int c = 0; c < 4; ++c) CHECK(a[c] == b[c]);
            }
        }

    // 3. random chains: an ordered scan of position functions gives every
    //    position's carry-in, as sequential propagation does
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 2000; ++trial) {
        const int len = 1 + (int)(rng() % 300);
        std::vector<uint64_t> s(len);
        for (auto& v : s) {
            const uint64_t hi = rng() % 4;
            uint32_t lo = (uint32_t)rng();
            if (rng() % 2) lo = 0xFFFFFFFFu - (uint32_t)(rng() % 6);
            v = hi * (1ull << 32) + lo;
            if (v > 4 * (1ull << 32) - 4) v = 4 * (1ull << 32) - 4;
        }
        const uint32_t cin = (uint32_t)(rng() % 4);
        uint32_t carry = cin, prefix = kCarryIdentity;
        for (int k = 0; k < len; ++k) {
            CHECK(carry_apply(prefix, cin) == carry);        // carry into position k
            const uint64_t t = s[k] + carry;
            carry = (uint32_t)(t >> 32);
            prefix = carry_compose(prefix, carry_fn_of_sum(s[k]));
        }
        CHECK(carry_apply(prefix, cin) == carry);
        // the same total by a pairwise tree
        std::vector<uint32_t> level(len);
        for (int k = 0; k < len; ++k) level[k] = carry_fn_of_sum(s[k]);
        while (level.size() > 1) {
            std::vector<uint32_t> next;
            for (size_t k = 0; k + 1 < level.size(); k += 2) next.push_back(carry_compose(level[k], level[k + 1]));
            if (level.size() % 2) next.push_back(level.back());
            level.swap(next);
        }
        CHECK(carry_apply(level[0], cin) == carry);
    }
    if (fails) {
        fprintf(stderr, "%d failures\n", fails);
        return 1;
    }
    printf("ok %zu functions\n", fs.size());
    return 0;
}
