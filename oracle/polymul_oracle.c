/*
 * CPU oracle for exact multiplication in Z_q[x]/(x^n + 1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  It is built into its
 * own shared library (liboracle.so), shares no header, source, table or helper
 * with the GPU library, and only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.
 *
 * What it computes (paper, Sec. 2.1, coefficient representation, and Sec. 2.2,
 * the fold rule and Eq. (3)):  the integer product of a(x) and b(x) in Z[x]
 * has degree at most 2n-2; folding every term of degree d >= n onto degree
 * d-n with a minus sign (x^n = -1) and reducing each coefficient mod q gives
 *
 *     c_j = ( sum_{i=0}^{j} a_i b_{j-i}  -  sum_{i=j+1}^{n-1} a_i b_{n+j-i} ) mod q,
 *
 * returned as the least non-negative residue in [0, q).  Input words are first
 * reduced mod q (coefficients are elements of Z_q, Eq. (1)).  n may be any
 * integer >= 1 here (Example 1 uses n = 3); q >= 2, prime or not (Sec. 2.1).
 *
 * Arithmetic is exact: the positive and the negative sums are accumulated
 * separately in unsigned 128-bit (32-bit q) or 192-bit (64-bit q) integers and
 * reduced once at the end.  No Montgomery/Barrett/NTT tricks appear here.
 *
 * RNS form (Sec. 2.4): a residue-number-system product is the same definition
 * applied independently to each residue channel with its own modulus.
 *
 * Cyclic ring Z_q[x]/(x^n - 1) (Sec. 2.1 names it as the other common ring):
 * there x^n = +1, so the folded terms are added instead of subtracted:
 *     c_j = ( sum_{i<=j} a_i b_{j-i} + sum_{i>j} a_i b_{n+j-i} ) mod q.
 */
#include <omp.h>
#include <stdint.h>
#include <stddef.h>

typedef unsigned __int128 u128;

/* (hi * 2^128 + lo) mod q for a 64-bit q, by the definition of the residue. */
static uint64_t mod_u192(uint64_t hi, u128 lo, uint64_t q) {
    u128 two64 = ((u128)1 << 64) % q;           /* 2^64 mod q */
    u128 two128 = (two64 * two64) % q;          /* 2^128 mod q */
    u128 r = ((u128)(hi % q) * two128) % q;
    r = (r + lo % q) % q;
    return (uint64_t)r;
}

/* One coefficient c_j of one product, 32-bit modulus; cyclic adds the folded terms. */
static uint32_t coeff_u32_ring(const uint32_t* a, const uint32_t* b, uint64_t n, uint32_t q, uint64_t j, int cyclic) {
    u128 pos = 0, neg = 0;
    for (uint64_t i = 0; i <= j; ++i)
        pos += (u128)((uint64_t)(a[i] % q) * (uint64_t)(b[j - i] % q));
    for (uint64_t i = j + 1; i < n; ++i)
        neg += (u128)((uint64_t)(a[i] % q) * (uint64_t)(b[n + j - i] % q));
    uint64_t p = (uint64_t)(pos % q), m = (uint64_t)(neg % q);
    if (cyclic) return (uint32_t)((p + m) % q);
    return (uint32_t)((p + q - m) % q);
}

static uint32_t coeff_u32(const uint32_t* a, const uint32_t* b, uint64_t n, uint32_t q, uint64_t j) {
    return coeff_u32_ring(a, b, n, q, j, 0);
}

/* One coefficient c_j of one product, 64-bit modulus: 192-bit accumulators;
   cyclic adds the folded terms. */
static uint64_t coeff_u64_ring(const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q, uint64_t j,
                               int cyclic) {
    u128 pos = 0, neg = 0;
    uint64_t pos_hi = 0, neg_hi = 0;
    for (uint64_t i = 0; i <= j; ++i) {
        u128 t = (u128)(a[i] % q) * (u128)(b[j - i] % q);
        pos += t;
        if (pos < t) ++pos_hi;
    }
    for (uint64_t i = j + 1; i < n; ++i) {
        u128 t = (u128)(a[i] % q) * (u128)(b[n + j - i] % q);
        neg += t;
        if (neg < t) ++neg_hi;
    }
    uint64_t p = mod_u192(pos_hi, pos, q), m = mod_u192(neg_hi, neg, q);
    if (cyclic) return (uint64_t)(((u128)p + m) % q);
    return (uint64_t)(((u128)p + q - m) % q);
}

static uint64_t coeff_u64(const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q, uint64_t j) {
    return coeff_u64_ring(a, b, n, q, j, 0);
}

/* c[batch][n] = a[batch][n] * b[batch][n] in Z_q[x]/(x^n+1), q < 2^32.
   Returns 0 on success, -1 on invalid arguments. */
int oracle_negacyclic_u32(const uint32_t* a, const uint32_t* b, uint32_t* c,
                          uint64_t n, uint32_t q, uint64_t batch) {
    if (n < 1 || q < 2 || !a || !b || !c) return -1;
    int64_t total = (int64_t)(batch * n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < total; ++k) {
        uint64_t p = (uint64_t)k / n, j = (uint64_t)k % n;
        c[p * n + j] = coeff_u32(a + p * n, b + p * n, n, q, j);
    }
    return 0;
}

/* Same for q < 2^64 with 64-bit words. */
int oracle_negacyclic_u64(const uint64_t* a, const uint64_t* b, uint64_t* c,
                          uint64_t n, uint64_t q, uint64_t batch) {
    if (n < 1 || q < 2 || !a || !b || !c) return -1;
    int64_t total = (int64_t)(batch * n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < total; ++k) {
        uint64_t p = (uint64_t)k / n, j = (uint64_t)k % n;
        c[p * n + j] = coeff_u64(a + p * n, b + p * n, n, q, j);
    }
    return 0;
}

/* c[batch][n] = a[batch][n] * b[batch][n] in Z_q[x]/(x^n-1), q < 2^32. */
int oracle_cyclic_u32(const uint32_t* a, const uint32_t* b, uint32_t* c,
                      uint64_t n, uint32_t q, uint64_t batch) {
    if (n < 1 || q < 2 || !a || !b || !c) return -1;
    int64_t total = (int64_t)(batch * n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < total; ++k) {
        uint64_t p = (uint64_t)k / n, j = (uint64_t)k % n;
        c[p * n + j] = coeff_u32_ring(a + p * n, b + p * n, n, q, j, 1);
    }
    return 0;
}

/* Same for q < 2^64 with 64-bit words. */
int oracle_cyclic_u64(const uint64_t* a, const uint64_t* b, uint64_t* c,
                      uint64_t n, uint64_t q, uint64_t batch) {
    if (n < 1 || q < 2 || !a || !b || !c) return -1;
    int64_t total = (int64_t)(batch * n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < total; ++k) {
        uint64_t p = (uint64_t)k / n, j = (uint64_t)k % n;
        c[p * n + j] = coeff_u64_ring(a + p * n, b + p * n, n, q, j, 1);
    }
    return 0;
}

/* RNS form: a, b, c are [batch][L][n]; channel l uses modulus q[l]. */
int oracle_negacyclic_rns_u32(const uint32_t* a, const uint32_t* b, uint32_t* c,
                              uint64_t n, const uint32_t* q, uint32_t L, uint64_t batch) {
    if (n < 1 || L < 1 || !q || !a || !b || !c) return -1;
    for (uint32_t l = 0; l < L; ++l)
        if (q[l] < 2) return -1;
    int64_t total = (int64_t)(batch * L * n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < total; ++k) {
        uint64_t pl = (uint64_t)k / n, j = (uint64_t)k % n;
        uint32_t l = (uint32_t)(pl % L);
        c[pl * n + j] = coeff_u32(a + pl * n, b + pl * n, n, q[l], j);
    }
    return 0;
}

/* Selected coefficients only: c_out[s] = c_{jidx[s]} of product pidx[s].
   Lets a test check a full-size workload on a sample of outputs. */
int oracle_negacyclic_u32_sample(const uint32_t* a, const uint32_t* b, uint64_t n, uint32_t q,
                                 const uint64_t* pidx, const uint64_t* jidx, uint64_t count,
                                 uint32_t* c_out) {
    if (n < 1 || q < 2 || !a || !b || !c_out) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < (int64_t)count; ++s)
        c_out[s] = coeff_u32(a + pidx[s] * n, b + pidx[s] * n, n, q, jidx[s] % n);
    return 0;
}

int oracle_negacyclic_u64_sample(const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q,
                                 const uint64_t* pidx, const uint64_t* jidx, uint64_t count,
                                 uint64_t* c_out) {
    if (n < 1 || q < 2 || !a || !b || !c_out) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < (int64_t)count; ++s)
        c_out[s] = coeff_u64(a + pidx[s] * n, b + pidx[s] * n, n, q, jidx[s] % n);
    return 0;
}

/* Threads the OpenMP loops above use from now on (a timing knob; results do not
   depend on it).  Returns the previous count. */
int oracle_set_threads(int threads) {
    const int prev = omp_get_max_threads();
    if (threads > 0) omp_set_num_threads(threads);
    return prev;
}
