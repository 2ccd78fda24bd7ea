/*
 * polymul.h -- exact multiplication in Z_q[x]/(x^n + 1) on gfx950 int8 MFMA.
 *
 * The operation (paper Sec. 2.1, Eq. (1) coefficient form; Sec. 2.2 fold rule
 * and Eq. (3)):  given a(x), b(x) with coefficients a_i, b_i in Z_q, return
 *
 *     c_j = ( sum_{i<=j} a_i b_{j-i} - sum_{i>j} a_i b_{n+j-i} ) mod q,   0 <= j < n,
 *
 * as the least non-negative residue.  The library computes it as a dense
 * integer matrix product (Sec. 2.2: one operand becomes the negacyclic
 * Toeplitz matrix of Eq. (3)), split into balanced signed 8-bit limbs
 * (Sec. 2.4, strategy (ii): several small units per coefficient) and tiled
 * over the degree (Sec. 2.5, divide and conquer).
 *
 * Conventions shared by every entry point:
 *   - Polynomials are stored lowest degree first, one machine word per
 *     coefficient (uint32_t for q < 2^32, uint64_t for q < 2^64), products
 *     laid out back to back: element [p][j] is at offset p*n + j.
 *   - a, b, c are DEVICE pointers owned by the caller, 16-byte aligned.  The
 *     library never frees or retains them (plans keep the pointers they were
 *     given).
 *   - Input words are read mod q (any 32/64-bit value is accepted); outputs
 *     are canonical, in [0, q).
 *   - n must be a power of two, 1 <= n <= 65536; q >= 2 (prime or not).
 *   - c must not overlap a or b (every output reads all of a and b).
 *   - Every call is asynchronous on `stream` (0 = the null stream).  Argument
 *     errors are returned before any HIP call is made; launch errors are
 *     reported as POLYMUL_EDEVICE.  No exception crosses this interface.
 *   - batch == 0 (or count == 0) is a successful no-op.
 *   - Stateless calls are thread-safe.
 */
#ifndef POLYMUL_H
#define POLYMUL_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    POLYMUL_OK = 0,
    POLYMUL_EINVAL = 1,        /* bad n, q, L, count, null pointer or size overflow */
    POLYMUL_EALIAS = 2,        /* c overlaps a or b */
    POLYMUL_EUNSUPPORTED = 3,  /* valid arguments outside what this library implements */
    POLYMUL_ENOMEM = 4,        /* device or host allocation failed (plans only) */
    POLYMUL_EDEVICE = 5,       /* a HIP call or kernel launch failed */
    POLYMUL_ESCRATCH = 6       /* needs more than the library's own scratch (allocation-free call) */
} polymul_status;

/* Human-readable name of a status code (static storage, never NULL). */
const char* polymul_status_string(polymul_status s);

/*
 * c[p] = a[p] * b[p] in Z_q[x]/(x^n+1) for p < batch, q < 2^32.
 * Paper Sec. 2.2 (Eq. (3)) for one pair; a batch of independent pairs is the
 * independent-instance parallelism of Sec. 2.4.
 * a, b, c: device, uint32_t[batch][n].
 */
polymul_status polymul_negacyclic(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                  uint64_t n, uint32_t q, uint64_t batch, hipStream_t stream);

/*
 * Same for a 64-bit modulus, q < 2^64 (for example 2^64 - 2^32 + 1).
 * a, b, c: device, uint64_t[batch][n].
 */
polymul_status polymul_negacyclic_u64(const uint64_t* a, const uint64_t* b, uint64_t* c,
                                      uint64_t n, uint64_t q, uint64_t batch, hipStream_t stream);

/*
 * RNS form (paper Sec. 2.4): each coefficient is held as its residues modulo
 * L moduli q[0..L-1]; the product is computed independently per residue
 * channel and the result stays in RNS (no CRT reconstruction).
 * a, b, c: device, uint32_t[batch][L][n]; channel l is reduced mod q[l].
 * q: HOST array of L moduli (each >= 2, < 2^32), copied during the call.
 */
polymul_status polymul_negacyclic_rns(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                      uint64_t n, const uint32_t* q, uint32_t L,
                                      uint64_t batch, hipStream_t stream);

/*
 * Cyclic ring Z_q[x]/(x^n - 1), the other ring the paper names (Sec. 2.1;
 * Sec. 2.5 notes the method adapts to it): x^n = +1, so the wrapped terms of
 * the matrix form keep their sign.  Same arguments, layout and errors as
 * polymul_negacyclic / polymul_negacyclic_u64.
 */
polymul_status polymul_cyclic(const uint32_t* a, const uint32_t* b, uint32_t* c,
                              uint64_t n, uint32_t q, uint64_t batch, hipStream_t stream);
polymul_status polymul_cyclic_u64(const uint64_t* a, const uint64_t* b, uint64_t* c,
                                  uint64_t n, uint64_t q, uint64_t batch, hipStream_t stream);

/*
 * The same product as polymul_negacyclic computed with plain 32x32->64-bit
 * integer multiply-adds (schoolbook, no matrix units).  A comparison baseline
 * for the MFMA path; never used as a fallback.
 */
polymul_status polymul_negacyclic_plain(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                        uint64_t n, uint32_t q, uint64_t batch, hipStream_t stream);

/*
 * Grouped products of uneven size in one persistent launch, replayed from a
 * HIP graph (paper Sec. 2.6-2.7: parameters fixed once per configuration,
 * Algorithm 1's GenConfig/ExtractDimensions done at plan time).  All 32-bit
 * groups share one persistent launch that takes work items largest first from
 * an atomic queue; 64-bit groups add one streaming launch each to the graph.
 *
 * Group g holds `count` independent products of degree bound n over Z_q:
 *   a, b, c: device, count*n words of elem_bytes (4: q < 2^32; 8: q < 2^64).
 * polymul_plan_create copies the group table, builds and uploads the work
 * list and captures the graph; the plan owns only that device work list, its
 * queue counters (left at zero by every launch), the graph and, when it cuts
 * large items along K into runs (items that would take more than an even share
 * of the work), the buffer the runs leave their residues in and the table of
 * the sums that one more launch forms from them.  Pointers are baked in: later executes read
 * and write the same buffers.  A plan must not be executed concurrently with
 * itself.  flags: 0, or POLYMUL_PLAN_NO_GRAPH to launch directly each time.
 */
typedef struct {
    const void* a;
    const void* b;
    void* c;
    uint64_t n;
    uint64_t q;
    uint64_t count;
    uint32_t elem_bytes;
} polymul_group;

typedef struct polymul_plan polymul_plan;

#define POLYMUL_PLAN_NO_GRAPH 1u

polymul_status polymul_plan_create(polymul_plan** plan, const polymul_group* groups,
                                   uint32_t ngroups, uint32_t flags);
polymul_status polymul_plan_execute(polymul_plan* plan, hipStream_t stream);
polymul_status polymul_plan_destroy(polymul_plan* plan);

/*
 * The paper's coefficient method (Sec. 2.4 RNS, Sec. 2.6 RNS base selection,
 * Algorithm 1): every coefficient is lifted to its centred integer in
 * (-q/2, q/2] and represented by its residues modulo co-prime moduli of at
 * most 8 bits, taken largest first until their product M exceeds
 * 2 n floor(q/2)^2 (1 + 2^-16) -- twice the largest possible |negacyclic sum|,
 * so the signed sums are recovered exactly.  Each modulus is one int8 matrix
 * product of centred residues (int32 sums, one MFMA per modulus per K-step);
 * the Chinese remainder theorem rebuilds each sum and reduces it mod q.  Same
 * results as polymul_negacyclic / polymul_negacyclic_rns, word for word.
 *
 * Arguments, layout and errors as polymul_negacyclic / polymul_negacyclic_rns;
 * n <= 4096 (the residue planes of both operands live in LDS), else
 * POLYMUL_EUNSUPPORTED.  Speed: at n = 4096 (one product's four output tiles share
 * their operand fragments in 2 x 2) this route runs 1.1x the limb route; below, each
 * product is a single output tile, every MFMA reads its own fragments and the
 * channels' planes leave one workgroup per CU, and the limb route is much faster
 * (n = 1024: about 7x, n = 512: about 14x).
 */
polymul_status polymul_negacyclic_crt(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                      uint64_t n, uint32_t q, uint64_t batch, hipStream_t stream);
polymul_status polymul_negacyclic_rns_crt(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                          uint64_t n, const uint32_t* q, uint32_t L,
                                          uint64_t batch, hipStream_t stream);
/*
 * The small moduli polymul_negacyclic_crt uses for degree bound n and modulus
 * q (Algorithm 1's ExtractModuli), largest first; `moduli` must hold 11
 * entries.  Host only, no HIP call.  EINVAL: bad n or q, null pointers.
 */
polymul_status polymul_crt_moduli(uint64_t n, uint32_t q, uint32_t* moduli, uint32_t* count);

/*
 * One operand shared by the whole batch (paper Sec. 2.2: one fixed matrix
 * times many vectors is a single matrix product; Sec. 4, fine-tuning (i): keep
 * one operand fixed so that what was prepared for it is reused).  Computes
 * c[i] = a[i] * b mod (x^n + 1, q) for every i: b's digit rows are staged
 * once per workgroup and reused for a chunk of products, only a[i] is staged
 * per product.  Same results as polymul_negacyclic with b repeated.
 *
 *   a, c: device, [batch][n] words (RNS: [batch][L][n], channel l mod q[l]).
 *   b:    device, [n] words (RNS: [L][n], one b per channel).
 *   c must not overlap a or b; a and b may overlap each other.
 * Other arguments, alignment and errors as for polymul_negacyclic /
 * polymul_negacyclic_rns / polymul_negacyclic_u64.
 */
polymul_status polymul_negacyclic_shared(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                         uint64_t n, uint32_t q, uint64_t batch, hipStream_t stream);
polymul_status polymul_negacyclic_rns_shared(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                             uint64_t n, const uint32_t* q, uint32_t L,
                                             uint64_t batch, hipStream_t stream);
polymul_status polymul_negacyclic_u64_shared(const uint64_t* a, const uint64_t* b, uint64_t* c,
                                             uint64_t n, uint64_t q, uint64_t batch, hipStream_t stream);

/*
 * Karatsuba's three-for-four trade (paper Sec. 4, the Karatsuba paragraph) on
 * top of the matrix product.  The paper splits each operand into a low and a
 * high half; in Z_q[x]/(x^n+1) this library splits into even and odd halves
 * instead, a(x) = a_e(x^2) + x a_o(x^2), because the halves then live in
 * Z_q[z]/(z^(n/2)+1), a ring of the same kind, and
 *   c_e = a_e b_e + z a_o b_o,   c_o = (a_e + a_o)(b_e + b_o) - a_e b_e - a_o b_o.
 * `depth` levels of this turn one product of degree bound n into 3^depth
 * products of degree bound n / 2^depth, which run on the same matrix kernels;
 * additions and subtractions are done mod q in two element-wise kernels.  The
 * result equals polymul_negacyclic_rns's word for word.
 *
 *   a, b, c, n, q, L, batch: as for polymul_negacyclic_rns (L <= 16; L <= 8
 *                when n / 2^depth > 8192).
 *   depth:       1, 2 or 3, with n / 2^depth >= 4; or 0 for the tuned choice
 *                for this degree bound and number of products (batch * L):
 *                polymul_tune_set_karatsuba, else a built-in one.  Where that
 *                choice is the direct route (no levels) the call is
 *                polymul_negacyclic_rns and the workspace is not used.
 *   workspace:   device, 16-byte aligned, at least
 *                polymul_karatsuba_workspace_size(...) bytes, owned by the
 *                caller, not overlapping a, b or c; its contents on entry do
 *                not matter and on return are unspecified.  Two calls that
 *                share a workspace must be ordered on one stream.
 * Errors: EINVAL for bad sizes, depth, moduli or a too small or misaligned
 * workspace; EALIAS for overlaps; EUNSUPPORTED for L > 8 with
 * n / 2^depth > 8192.  No memory is allocated.
 */
polymul_status polymul_karatsuba_workspace_size(uint64_t n, uint32_t L, uint64_t batch,
                                                uint32_t depth, uint64_t* bytes);
/*
 * The same route for 64-bit words and one modulus q < 2^64 (a, b, c as for
 * polymul_negacyclic_u64): the sub-products run on the K-streaming kernel,
 * their K range cut into up to four runs (POLYMUL_TUNE_U64_KARATSUBA_RUNS) when
 * that fills the GPU's rounds of workgroups better.  depth 0 takes the tuned
 * choice for (n, batch) as above, the direct polymul_negacyclic_u64 included.  Workspace rules and errors as above, sized by
 * polymul_karatsuba_u64_workspace_size (room for the runs included).
 */
polymul_status polymul_karatsuba_u64_workspace_size(uint64_t n, uint64_t batch, uint32_t depth,
                                                    uint64_t* bytes);
polymul_status polymul_negacyclic_u64_karatsuba(const uint64_t* a, const uint64_t* b, uint64_t* c,
                                                uint64_t n, uint64_t q, uint64_t batch,
                                                uint32_t depth, void* workspace,
                                                uint64_t workspace_bytes, hipStream_t stream);
polymul_status polymul_negacyclic_rns_karatsuba(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                                uint64_t n, const uint32_t* q, uint32_t L,
                                                uint64_t batch, uint32_t depth, void* workspace,
                                                uint64_t workspace_bytes, hipStream_t stream);

/*
 * polymul_negacyclic_rns_karatsuba for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the workspace is not an argument but a buffer of
 * POLYMUL_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on,
 * set aside when the library's code is loaded on that GPU and kept until the
 * process ends.  The call itself allocates nothing.
 *   a, b, c, n, q, L, batch, depth: as for polymul_negacyclic_rns_karatsuba;
 *   same results, word for word.
 * Every call on one GPU uses that GPU's one buffer: calls that may overlap in
 * time on one GPU (unordered streams, host threads) race and give wrong results;
 * order them on one stream.  The buffer's contents on entry do not matter.
 * Errors: as polymul_negacyclic_rns_karatsuba, and POLYMUL_ESCRATCH when the
 * call needs more than POLYMUL_NOALLOC_SCRATCH_BYTES of workspace (as sized by
 * polymul_karatsuba_workspace_size); split such a batch.
 */
#define POLYMUL_NOALLOC_SCRATCH_BYTES (64ull << 20)
polymul_status polymul_negacyclic_rns_karatsuba_noalloc(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                                        uint64_t n, const uint32_t* q, uint32_t L,
                                                        uint64_t batch, uint32_t depth, hipStream_t stream);

/*
 * Tile table of the LDS-resident 32-bit path (paper Sec. 2.6, matrix dimension
 * selection: the best block size is found by experiment).  For degree bound n
 * and limb count L (1..4), t is the side of the Toeplitz tiles the product is
 * cut into (n = t * r): n itself when n <= 32, otherwise a power of two in
 * [32, min(n, 128)] (32x32 output tiles, v_mfma_i32_32x32x32_i8), or 16 for
 * 64 <= n <= 512 (16x16 output tiles, v_mfma_i32_16x16x64_i8, the built-in
 * choice there).  t = 0 restores the built-in choice.  The table is
 * process-wide; the autotuner (paper_2307_06554_amd/tune.py) times the
 * candidates on the GPU and calls polymul_tune_set with the winners.  Takes
 * effect for launches and plans created afterwards.  No HIP call is made.
 * EINVAL: bad n, L or t; EUNSUPPORTED: the tile does not fit in LDS.
 */
polymul_status polymul_tune_set(uint64_t n, uint32_t L, uint32_t t);
polymul_status polymul_tune_get(uint64_t n, uint32_t L, uint32_t* t);

/*
 * Process-wide scheduling knobs of grouped plans (paper Sec. 2.6: parameters
 * found by experiment), read when a plan is created; results never depend on
 * them.  No HIP call is made.  EINVAL: unknown parameter or value out of range.
 *   POLYMUL_TUNE_PLAN_SHARE_PCT (10..1000, default 140): items estimated to take
 *     longer than this percentage of a CU's even share of the plan's work have
 *     their K range cut into runs.
 *   POLYMUL_TUNE_PLAN_STREAM_PCT (50..400, default 125): weight of a K-streamed
 *     block's matrix work against a resident group's in those estimates.
 *   POLYMUL_TUNE_U64_KARATSUBA_RUNS (1, 2 or 4, default 4): most K runs the
 *     64-bit Karatsuba route cuts its streamed sub-products into.
 */
#define POLYMUL_TUNE_PLAN_SHARE_PCT 1u
#define POLYMUL_TUNE_PLAN_STREAM_PCT 2u
#define POLYMUL_TUNE_U64_KARATSUBA_RUNS 3u
polymul_status polymul_tune_param_set(uint32_t param, uint64_t value);
polymul_status polymul_tune_param_get(uint32_t param, uint64_t* value);

/*
 * Karatsuba depth table (paper Sec. 4, Karatsuba; Sec. 2.6, parameters by
 * experiment): the depth that depth 0 resolves to for degree bound n and calls
 * of `products` products (batch * L for the RNS route, batch for the 64-bit
 * route; bucketed by floor(log2 products)), for 32-bit (elem_bytes 4) or 64-bit
 * (8) words.  depth 0 = the direct route, 1..3 = levels, 0xFF = back to the
 * built-in choice.  The get call returns the depth in force.  No HIP call.
 * EINVAL: bad n, products, elem_bytes or depth.
 */
polymul_status polymul_tune_set_karatsuba(uint64_t n, uint64_t products, uint32_t elem_bytes, uint32_t depth);
polymul_status polymul_tune_get_karatsuba(uint64_t n, uint64_t products, uint32_t elem_bytes, uint32_t* depth);


#ifdef __cplusplus
}
#endif

#endif /* POLYMUL_H */
