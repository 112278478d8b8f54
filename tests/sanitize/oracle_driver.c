/*
 * Runs the CPU oracle (oracle/oracle.c) over seeded random inputs so that a
 * sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer) sees every
 * function on every key type and order, empty sides included: the merge,
 * the brute-force co-rank and Algorithm 1 for every rank, and the
 * segmented merge.  It also checks what must hold whatever the inputs: the
 * two co-rank routines agree, and the merge output is ordered.  Exit status
 * 0 when all of that holds.  Test infrastructure only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_stable_merge(int kt, const void *A, const uint32_t *Av, uint64_t m, const void *B,
                         const uint32_t *Bv, uint64_t n, void *C, uint32_t *Cv);
uint64_t oracle_co_rank_brute(int kt, uint64_t i, const void *A, uint64_t m, const void *B, uint64_t n);
int oracle_co_rank_alg1(int kt, uint64_t i, const void *A, uint64_t m, const void *B, uint64_t n,
                        uint64_t *j_out, uint64_t *k_out, uint64_t *trace, uint64_t trace_cap,
                        uint64_t *n_states, uint64_t *iters);
void oracle_stable_merge_segmented(int kt, const void *A, const uint32_t *Av, const uint64_t *a_off,
                                   const void *B, const uint32_t *Bv, const uint64_t *b_off,
                                   uint64_t num_seg, void *C, uint32_t *Cv);
int oracle_key_size(int kt);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint64_t next(void) {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

/* n sorted keys of type kt (ascending for 0-2, descending for 3-5) drawn
 * from an alphabet of `alpha` values. */
static void *sorted_keys(int kt, uint64_t n, uint64_t alpha) {
    const int ks = oracle_key_size(kt);
    void *p = malloc(n ? n * ks : 1);
    uint64_t v = 0;
    for (uint64_t x = 0; x < n; x++) {
        if (next() % 3 == 0) v += 1 + next() % 2;
        const uint64_t c = v < alpha ? v : alpha; /* nondecreasing, at most alpha */
        const uint64_t val = kt >= 3 ? alpha - c : c;
        if (ks == 8)
            ((uint64_t *)p)[x] = val;
        else if (kt % 3 == 2)
            ((float *)p)[x] = (float)val - (float)(alpha / 2);
        else
            ((uint32_t *)p)[x] = (uint32_t)val;
    }
    return p;
}

static int ordered(int kt, const void *C, uint64_t N) {
    for (uint64_t x = 1; x < N; x++) {
        int bad;
        switch (kt % 3) {
            case 0: bad = ((const uint32_t *)C)[x - 1] > ((const uint32_t *)C)[x]; break;
            case 1: bad = ((const uint64_t *)C)[x - 1] > ((const uint64_t *)C)[x]; break;
            default: bad = ((const float *)C)[x - 1] > ((const float *)C)[x]; break;
        }
        if (kt >= 3) {
            switch (kt % 3) {
                case 0: bad = ((const uint32_t *)C)[x - 1] < ((const uint32_t *)C)[x]; break;
                case 1: bad = ((const uint64_t *)C)[x - 1] < ((const uint64_t *)C)[x]; break;
                default: bad = ((const float *)C)[x - 1] < ((const float *)C)[x]; break;
            }
        }
        if (bad) return 0;
    }
    return 1;
}

int main(void) {
    int failures = 0;
    for (int kt = 0; kt < 6; kt++) {
        for (int rep = 0; rep < 40; rep++) {
            const uint64_t m = next() % 60, n = next() % 60, alpha = 1 + next() % 8;
            void *A = sorted_keys(kt, m, alpha), *B = sorted_keys(kt, n, alpha);
            const int ks = oracle_key_size(kt);
            uint32_t *Av = malloc((m ? m : 1) * 4), *Bv = malloc((n ? n : 1) * 4);
            for (uint64_t x = 0; x < m; x++) Av[x] = (uint32_t)x;
            for (uint64_t y = 0; y < n; y++) Bv[y] = 0x80000000u | (uint32_t)y;
            void *C = malloc((m + n ? m + n : 1) * ks);
            uint32_t *Cv = malloc((m + n ? m + n : 1) * 4);
            oracle_stable_merge(kt, A, Av, m, B, Bv, n, C, Cv);
            if (!ordered(kt, C, m + n)) failures++;
            oracle_stable_merge(kt, A, NULL, m, B, NULL, n, C, NULL);
            uint64_t trace[4 * 140];
            for (uint64_t i = 0; i <= m + n; i++) {
                uint64_t j, k, states, iters;
                const uint64_t jb = oracle_co_rank_brute(kt, i, A, m, B, n);
                if (oracle_co_rank_alg1(kt, i, A, m, B, n, &j, &k, trace, 140, &states, &iters) != 0 ||
                    j != jb || j + k != i)
                    failures++;
            }
            free(A); free(B); free(Av); free(Bv); free(C); free(Cv);
        }
        /* segmented: empty segments and empty sides among them */
        const uint64_t S = 1 + next() % 20;
        uint64_t *a_off = malloc((S + 1) * 8), *b_off = malloc((S + 1) * 8);
        a_off[0] = b_off[0] = 0;
        for (uint64_t s = 0; s < S; s++) {
            a_off[s + 1] = a_off[s] + next() % 7;
            b_off[s + 1] = b_off[s] + next() % 7;
        }
        const uint64_t ta = a_off[S], tb = b_off[S];
        void *A = sorted_keys(kt, ta, 5), *B = sorted_keys(kt, tb, 5);
        uint32_t *Av = calloc(ta ? ta : 1, 4), *Bv = calloc(tb ? tb : 1, 4);
        void *C = malloc((ta + tb ? ta + tb : 1) * oracle_key_size(kt));
        uint32_t *Cv = malloc((ta + tb ? ta + tb : 1) * 4);
        oracle_stable_merge_segmented(kt, A, Av, a_off, B, Bv, b_off, S, C, Cv);
        free(A); free(B); free(Av); free(Bv); free(C); free(Cv); free(a_off); free(b_off);
    }
    printf("oracle driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
