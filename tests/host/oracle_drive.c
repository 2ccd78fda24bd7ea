/* Drives every entry point of the C oracle through small cases with known
 * answers, so that a sanitized build (address, undefined behaviour) walks all of
 * its code: Example 1's three coefficient formulas (paper Sec. 2.2), x^(n-1)
 * times x giving -1 (the ring's defining relation), multiplication by x^k as a
 * signed rotation, commutativity, all-(q-1) operands whose products are 1 mod q
 * (closed form c_j = 2j + 2 - n, through the 192-bit carries of the 64-bit path),
 * the cyclic ring's all-ones product, the RNS form channel by channel and the
 * sampled form.  Built and run by tests/test_host_arith.py; prints "ok <cases>". */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_negacyclic_u32(const uint32_t*, const uint32_t*, uint32_t*, uint64_t, uint32_t, uint64_t);
int oracle_negacyclic_u64(const uint64_t*, const uint64_t*, uint64_t*, uint64_t, uint64_t, uint64_t);
int oracle_cyclic_u32(const uint32_t*, const uint32_t*, uint32_t*, uint64_t, uint32_t, uint64_t);
int oracle_cyclic_u64(const uint64_t*, const uint64_t*, uint64_t*, uint64_t, uint64_t, uint64_t);
int oracle_negacyclic_rns_u32(const uint32_t*, const uint32_t*, uint32_t*, uint64_t, const uint32_t*, uint32_t,
                              uint64_t);
int oracle_negacyclic_u32_sample(const uint32_t*, const uint32_t*, uint64_t, uint32_t, const uint64_t*,
                                 const uint64_t*, uint64_t, uint32_t*);
int oracle_negacyclic_u64_sample(const uint64_t*, const uint64_t*, uint64_t, uint64_t, const uint64_t*,
                                 const uint64_t*, uint64_t, uint64_t*);

typedef unsigned __int128 u128;
static unsigned long long cases = 0;
static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }

#define CHECK(c, msg)                                                   \
    do {                                                                \
        ++cases;                                                        \
        if (!(c)) { fprintf(stderr, "FAIL line %d: %s\n", __LINE__, msg); exit(1); } \
    } while (0)

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }
static uint64_t addm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t subm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - b % q) % q); }

static void example1(uint64_t q) {
    uint64_t a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) { a[i] = rnd() % q; b[i] = rnd() % q; }
    uint64_t e0 = subm(subm(mulmod(a[0], b[0], q), mulmod(a[1], b[2], q), q), mulmod(a[2], b[1], q), q);
    uint64_t e1 = subm(addm(mulmod(a[0], b[1], q), mulmod(a[1], b[0], q), q), mulmod(a[2], b[2], q), q);
    uint64_t e2 = addm(addm(mulmod(a[0], b[2], q), mulmod(a[1], b[1], q), q), mulmod(a[2], b[0], q), q);
    if (q < (1ull << 32)) {
        uint32_t a32[3], b32[3], c32[3];
        for (int i = 0; i < 3; ++i) { a32[i] = (uint32_t)a[i]; b32[i] = (uint32_t)b[i]; }
        CHECK(oracle_negacyclic_u32(a32, b32, c32, 3, (uint32_t)q, 1) == 0, "u32 n=3");
        CHECK(c32[0] == e0 && c32[1] == e1 && c32[2] == e2, "Example 1, 32-bit");
    }
    CHECK(oracle_negacyclic_u64(a, b, c, 3, q, 1) == 0, "u64 n=3");
    CHECK(c[0] == e0 && c[1] == e1 && c[2] == e2, "Example 1, 64-bit");
}

static void ring_relations_u64(uint64_t n, uint64_t q) {
    uint64_t* a = calloc(n, 8); uint64_t* b = calloc(n, 8); uint64_t* c = calloc(n, 8); uint64_t* d = calloc(n, 8);
    /* x times x^(n-1) = -1 */
    a[1 % n] = 1; b[n - 1] = 1;
    if (n > 1) {
        CHECK(oracle_negacyclic_u64(a, b, c, n, q, 1) == 0, "x^n");
        CHECK(c[0] == q - 1, "x^n = -1");
        for (uint64_t j = 1; j < n; ++j) CHECK(c[j] == 0, "x^n = -1, other coefficients");
    }
    /* x^k a = signed rotation; commutativity */
    for (uint64_t i = 0; i < n; ++i) { a[i] = rnd() % q; b[i] = 0; }
    uint64_t k = rnd() % n;
    b[k] = 1;
    CHECK(oracle_negacyclic_u64(a, b, c, n, q, 1) == 0, "rotation");
    for (uint64_t j = 0; j < n; ++j) CHECK(c[j] == (j >= k ? a[j - k] : subm(0, a[n + j - k], q)), "rotation");
    for (uint64_t i = 0; i < n; ++i) b[i] = rnd() % q;
    CHECK(oracle_negacyclic_u64(a, b, c, n, q, 1) == 0 && oracle_negacyclic_u64(b, a, d, n, q, 1) == 0, "comm");
    CHECK(memcmp(c, d, n * 8) == 0, "commutativity");
    /* all q - 1: every product is 1 mod q, so c_j = (j + 1) - (n - 1 - j) mod q */
    for (uint64_t i = 0; i < n; ++i) a[i] = b[i] = q - 1;
    CHECK(oracle_negacyclic_u64(a, b, c, n, q, 1) == 0, "all q-1");
    for (uint64_t j = 0; j < n; ++j) {
        int64_t v = 2 * (int64_t)j + 2 - (int64_t)n;
        uint64_t want = v >= 0 ? (uint64_t)v % q : subm(0, (uint64_t)(-v) % q, q);
        CHECK(c[j] == want, "all q-1 closed form");
    }
    /* cyclic ring: all ones gives n everywhere */
    for (uint64_t i = 0; i < n; ++i) a[i] = b[i] = 1;
    CHECK(oracle_cyclic_u64(a, b, c, n, q, 1) == 0, "cyclic");
    for (uint64_t j = 0; j < n; ++j) CHECK(c[j] == n % q, "cyclic all ones");
    /* sampled form equals the full product */
    for (uint64_t i = 0; i < n; ++i) { a[i] = rnd(); b[i] = rnd(); }  /* non-canonical words */
    CHECK(oracle_negacyclic_u64(a, b, c, n, q, 1) == 0, "full");
    uint64_t pidx[8], jidx[8], out[8];
    for (int s = 0; s < 8; ++s) { pidx[s] = 0; jidx[s] = rnd() % n; }
    CHECK(oracle_negacyclic_u64_sample(a, b, n, q, pidx, jidx, 8, out) == 0, "sample");
    for (int s = 0; s < 8; ++s) CHECK(out[s] == c[jidx[s]], "sample equals full");
    free(a); free(b); free(c); free(d);
}

static void forms_u32(uint64_t n, uint32_t q, uint64_t batch) {
    uint32_t* a = malloc(batch * n * 4); uint32_t* b = malloc(batch * n * 4);
    uint32_t* c = malloc(batch * n * 4); uint32_t* d = malloc(batch * n * 4);
    uint64_t* a64 = malloc(batch * n * 8); uint64_t* b64 = malloc(batch * n * 8); uint64_t* c64 = malloc(batch * n * 8);
    for (uint64_t i = 0; i < batch * n; ++i) {
        a[i] = (uint32_t)rnd(); b[i] = (uint32_t)rnd();
        a64[i] = a[i]; b64[i] = b[i];
    }
    CHECK(oracle_negacyclic_u32(a, b, c, n, q, batch) == 0, "u32");
    CHECK(oracle_negacyclic_u64(a64, b64, c64, n, q, batch) == 0, "u64 same q");
    for (uint64_t i = 0; i < batch * n; ++i) CHECK(c[i] == c64[i], "32- and 64-bit forms agree");
    CHECK(oracle_cyclic_u32(a, b, c, n, q, batch) == 0, "cyclic u32");
    CHECK(oracle_cyclic_u64(a64, b64, c64, n, q, batch) == 0, "cyclic u64");
    for (uint64_t i = 0; i < batch * n; ++i) CHECK(c[i] == c64[i], "cyclic forms agree");
    /* RNS: channel l of [batch][2][n/2]-shaped data equals the plain product mod q_l */
    if (n % 2 == 0 && batch > 0) {
        uint32_t qs[2] = {q, q / 2 + 2};
        uint64_t m = n / 2;
        CHECK(oracle_negacyclic_rns_u32(a, b, c, m, qs, 2, batch) == 0, "rns");
        for (uint64_t p = 0; p < batch; ++p)
            for (int l = 0; l < 2; ++l) {
                const uint64_t off = (p * 2 + l) * m;
                CHECK(oracle_negacyclic_u32(a + off, b + off, d, m, qs[l], 1) == 0, "rns channel");
                CHECK(memcmp(c + off, d, m * 4) == 0, "rns channel equals the plain product");
            }
    }
    uint64_t pidx[8], jidx[8];
    uint32_t out[8];
    CHECK(oracle_negacyclic_u32(a, b, c, n, q, batch) == 0, "u32 again");
    for (int s = 0; s < 8; ++s) { pidx[s] = rnd() % batch; jidx[s] = rnd() % n; }
    CHECK(oracle_negacyclic_u32_sample(a, b, n, q, pidx, jidx, 8, out) == 0, "sample u32");
    for (int s = 0; s < 8; ++s) CHECK(out[s] == c[pidx[s] * n + jidx[s]], "sample u32 equals full");
    /* argument errors */
    CHECK(oracle_negacyclic_u32(a, b, c, 0, q, batch) == -1, "n = 0 rejected");
    CHECK(oracle_negacyclic_u32(a, b, c, n, 1, batch) == -1, "q = 1 rejected");
    CHECK(oracle_negacyclic_u64(NULL, b64, c64, n, q, batch) == -1, "null rejected");
    free(a); free(b); free(c); free(d); free(a64); free(b64); free(c64);
}

int main(void) {
    const uint64_t q64[] = {2, 3, 3329, 1068236801ull, 4294967291ull, 0xFFFFFFFF00000001ull, 0xFFFFFFFFFFFFFFC5ull,
                            (1ull << 63) + 2};
    for (size_t i = 0; i < sizeof(q64) / sizeof(q64[0]); ++i) {
        for (int r = 0; r < 20; ++r) example1(q64[i]);
        const uint64_t ns[] = {1, 2, 3, 4, 7, 16, 64, 257};
        for (size_t k = 0; k < sizeof(ns) / sizeof(ns[0]); ++k) ring_relations_u64(ns[k], q64[i]);
    }
    const uint32_t q32[] = {2, 17, 3329, 65537, 1068236801u, 4294967291u, 4294967295u};
    for (size_t i = 0; i < sizeof(q32) / sizeof(q32[0]); ++i) {
        forms_u32(64, q32[i], 3);
        forms_u32(5, q32[i], 2);
        forms_u32(1, q32[i], 4);
    }
    printf("ok %llu\n", cases);
    return 0;
}
