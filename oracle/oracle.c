/*
 * CPU oracle for the stable two-way merge and for co-ranking, after
 * C. Siebert and J. L. Traeff, "Perfectly load-balanced, optimal, stable,
 * parallel merge" (arXiv:1303.4312).
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it. It shares no source, header, table or helper with the GPU path,
 * and the GPU path never calls it.
 *
 * Everything here is plain, single-threaded and deliberately slow:
 *   - oracle_stable_merge: the sequential stable merge the paper assumes
 *     (Section 1) with its tie rule (Section 2: among equal keys, every
 *     element of A precedes every element of B, each side in input order).
 *   - oracle_co_rank_brute: the definition of the co-ranks of rank i
 *     (Section 2 and Lemma 1): run the merge for i outputs and count how
 *     many came from A.
 *   - oracle_co_rank_alg1: Algorithm 1 of Section 2, in the paper's order and
 *     notation, instrumented with a state trace and an iteration count.
 *   - oracle_stable_merge_segmented: the merge applied independently to each
 *     segment of a batch (not in the paper; each segment is one instance of
 *     the Section 2 problem).
 *
 * Key types: 0 = uint32, 1 = uint64, 2 = float32 (IEEE comparison, so -0.0
 * and +0.0 are equal keys; NaN is outside the paper's totally ordered key
 * model and must not occur).  Payloads, when present, are uint32 and travel
 * with their key.
 *
 * Parity pins: every function here is checked by the CPU tests against the
 * paper's worked example (Figures 1-3), exhaustive enumeration on tiny
 * inputs, closed forms and library routines; none is unpinned.
 */
#include <stdint.h>
#include <string.h>

#define ORACLE_U32 0
#define ORACLE_U64 1
#define ORACLE_F32 2
/* Types 3, 4, 5: the same keys under the reversed order (nonincreasing).
 * The method is stated for any total order on keys (Section 2), so these
 * merge with x <= y read as x >= y and keep the tie rule (A first). */
#define ORACLE_DESC 3

static int base_type(int kt) { return kt >= ORACLE_DESC ? kt - ORACLE_DESC : kt; }

/* x <= y for element a of A and element b of B in plain numeric order. */
static int num_le(int t, const void *A, uint64_t a, const void *B, uint64_t b)
{
    if (t == ORACLE_U32)
        return ((const uint32_t *)A)[a] <= ((const uint32_t *)B)[b];
    if (t == ORACLE_U64)
        return ((const uint64_t *)A)[a] <= ((const uint64_t *)B)[b];
    return ((const float *)A)[a] <= ((const float *)B)[b];
}

static int num_lt(int t, const void *A, uint64_t a, const void *B, uint64_t b)
{
    if (t == ORACLE_U32)
        return ((const uint32_t *)A)[a] < ((const uint32_t *)B)[b];
    if (t == ORACLE_U64)
        return ((const uint64_t *)A)[a] < ((const uint64_t *)B)[b];
    return ((const float *)A)[a] < ((const float *)B)[b];
}

/* A[a] <= B[b] under the key order. */
static int key_le(int kt, const void *A, uint64_t a, const void *B, uint64_t b)
{
    return kt >= ORACLE_DESC ? num_le(base_type(kt), B, b, A, a) : num_le(kt, A, a, B, b);
}

/* A[a] > B[b] and B[b] >= A[a] under the key order, spelled out as in
 * Algorithm 1's two tests. */
static int key_gt(int kt, const void *A, uint64_t a, const void *B, uint64_t b)
{
    return kt >= ORACLE_DESC ? num_lt(base_type(kt), A, a, B, b) : num_lt(kt, B, b, A, a);
}

static int key_ge(int kt, const void *A, uint64_t a, const void *B, uint64_t b)
{
    return kt >= ORACLE_DESC ? num_le(base_type(kt), A, a, B, b) : num_le(kt, B, b, A, a);
}

static size_t key_size(int kt) { return base_type(kt) == ORACLE_U64 ? 8 : 4; }

int oracle_key_size(int kt) { return (int)key_size(kt); }

/*
 * Sequential stable merge (Section 1; tie rule of Section 2).
 * Output o takes the next element of A when A is not exhausted and either B
 * is exhausted or A's next key is <= B's next key; otherwise it takes B's.
 * The "<=" is what puts equal A keys before equal B keys.
 * Av/Bv/Cv may all be NULL (keys only) or all non-NULL (key + payload).
 */
void oracle_stable_merge(int kt,
                         const void *A, const uint32_t *Av, uint64_t m,
                         const void *B, const uint32_t *Bv, uint64_t n,
                         void *C, uint32_t *Cv)
{
    size_t ks = key_size(kt);
    uint64_t a = 0, b = 0;
    for (uint64_t o = 0; o < m + n; o++) {
        int take_a = (a < m) && (b == n || key_le(kt, A, a, B, b));
        if (take_a) {
            memcpy((char *)C + o * ks, (const char *)A + a * ks, ks);
            if (Cv) Cv[o] = Av[a];
            a++;
        } else {
            memcpy((char *)C + o * ks, (const char *)B + b * ks, ks);
            if (Cv) Cv[o] = Bv[b];
            b++;
        }
    }
}

/*
 * Co-rank of rank i by definition (Section 2, Lemma 1): the prefix
 * C[0..i) of the stable merge is the stable merge of A[0..j) and B[0..k);
 * j is the number of outputs among the first i that come from A, k = i - j.
 * Runs the merge decisions for i steps without writing anything.
 * Requires 0 <= i <= m + n; returns j.
 */
uint64_t oracle_co_rank_brute(int kt, uint64_t i,
                              const void *A, uint64_t m,
                              const void *B, uint64_t n)
{
    uint64_t a = 0, b = 0;
    for (uint64_t o = 0; o < i; o++) {
        int take_a = (a < m) && (b == n || key_le(kt, A, a, B, b));
        if (take_a) a++; else b++;
    }
    return a;
}

/*
 * Algorithm 1 of Section 2: co_rank(i, A, m, B, n).
 *
 * State: j and k with j + k = i throughout, and lower bounds j_low and k_low.
 * Start with as many of the i outputs from A as possible (j = min(i, m)),
 * j_low = max(0, i - n) so that k can never pass n.  Each round tests the
 * first Lemma condition (j > 0, k < n and A[j-1] > B[k] means j is too big:
 * move half of the distance down to j_low over to k, and raise k_low to the
 * old k), else the second (k > 0, j < m and B[k-1] >= A[j] means k is too
 * big: move half of the distance down to k_low over to j, and raise j_low to
 * the old j), else stop.  Both tests are "conditional and": the key reads
 * happen only when the index guards hold, so no sentinel is ever read.
 *
 * k_low is not given a starting value in the paper; only the first
 * condition can fail in the first round, which assigns it before any read.
 * It is started at max(0, i - m) here, which the algorithm never reads.
 *
 * trace: if non-NULL, receives up to trace_cap states (j, k, j_low, k_low),
 * four uint64 each, starting with the initial state (k_low of the initial
 * state is written as UINT64_MAX: not yet defined).
 * *n_states receives the number of states visited (initial + one per
 * updating round), *iters the number of updating rounds.
 * Requires 0 <= i <= m + n.  Returns 0, or -1 if the rounds exceed 130
 * (impossible for correct code on 64-bit sizes: the search interval at
 * least halves every round), so that a broken variant cannot loop forever.
 */
int oracle_co_rank_alg1(int kt, uint64_t i,
                        const void *A, uint64_t m,
                        const void *B, uint64_t n,
                        uint64_t *j_out, uint64_t *k_out,
                        uint64_t *trace, uint64_t trace_cap,
                        uint64_t *n_states, uint64_t *iters)
{
    uint64_t j = i < m ? i : m;
    uint64_t k = i - j;
    uint64_t j_low = i > n ? i - n : 0;
    uint64_t k_low = i > m ? i - m : 0;
    int k_low_defined = 0;
    uint64_t states = 0, rounds = 0;
    int active = 1;

    if (trace && states < trace_cap) {
        trace[4 * states + 0] = j;
        trace[4 * states + 1] = k;
        trace[4 * states + 2] = j_low;
        trace[4 * states + 3] = UINT64_MAX;
    }
    states++;

    while (active) {
        if (j > 0 && k < n && key_gt(kt, A, j - 1, B, k)) {
            /* first Lemma condition violated: decrease j */
            uint64_t delta = (j - j_low + 1) / 2;
            k_low = k;
            k_low_defined = 1;
            j -= delta;
            k += delta;
        } else if (k > 0 && j < m && key_ge(kt, B, k - 1, A, j)) {
            /* second Lemma condition violated: decrease k */
            uint64_t delta = (k - k_low + 1) / 2;
            j_low = j;
            j += delta;
            k -= delta;
        } else {
            active = 0; /* both conditions hold: (j, k) found */
            continue;
        }
        rounds++;
        if (rounds > 130) return -1;
        if (trace && states < trace_cap) {
            trace[4 * states + 0] = j;
            trace[4 * states + 1] = k;
            trace[4 * states + 2] = j_low;
            trace[4 * states + 3] = k_low_defined ? k_low : UINT64_MAX;
        }
        states++;
    }
    *j_out = j;
    *k_out = k;
    if (n_states) *n_states = states;
    if (iters) *iters = rounds;
    return 0;
}

/*
 * Batch of independent merges.  Segment s merges A[a_off[s] .. a_off[s+1])
 * with B[b_off[s] .. b_off[s+1]) into C starting at a_off[s] + b_off[s].
 * Offsets have num_seg + 1 nondecreasing entries.
 */
void oracle_stable_merge_segmented(int kt,
                                   const void *A, const uint32_t *Av,
                                   const uint64_t *a_off,
                                   const void *B, const uint32_t *Bv,
                                   const uint64_t *b_off,
                                   uint64_t num_seg,
                                   void *C, uint32_t *Cv)
{
    size_t ks = key_size(kt);
    for (uint64_t s = 0; s < num_seg; s++) {
        uint64_t a0 = a_off[s], b0 = b_off[s];
        uint64_t c0 = a0 + b0;
        oracle_stable_merge(kt,
                            (const char *)A + a0 * ks, Av ? Av + a0 : NULL,
                            a_off[s + 1] - a0,
                            (const char *)B + b0 * ks, Bv ? Bv + b0 : NULL,
                            b_off[s + 1] - b0,
                            (char *)C + c0 * ks, Cv ? Cv + c0 : NULL);
    }
}
