/*
 * A C client of the library, with no Python: merges key + payload pairs on
 * the GPU through the C ABI (device pointers, a caller-owned workspace, a
 * stream), co-ranks on the device and on the host, and checks every result
 * against the oracle's C merge and brute-force co-rank (oracle/oracle.c,
 * linked into this test program).  Exit status 0 and "c client ok" on
 * success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "corank_merge.h"

#define ORACLE_U32 0 /* the oracle's code for uint32 keys */

void oracle_stable_merge(int kt, const void *A, const uint32_t *Av, uint64_t m, const void *B,
                         const uint32_t *Bv, uint64_t n, void *C, uint32_t *Cv);
uint64_t oracle_co_rank_brute(int kt, uint64_t i, const void *A, uint64_t m, const void *B,
                              uint64_t n);

#define HIP_OK(x)                                                              \
    do {                                                                       \
        if ((x) != hipSuccess) {                                               \
            fprintf(stderr, "HIP call failed at line %d\n", __LINE__);       \
            return 2;                                                          \
        }                                                                      \
    } while (0)

static uint64_t next(uint64_t *s) {  /* 64-bit LCG, upper bits */
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return *s >> 33;
}

/* sorted keys with runs of equal values: steps of 0..3 */
static void sorted_keys(uint32_t *k, uint64_t len, uint64_t seed) {
    uint64_t s = seed;
    uint32_t v = 0;
    for (uint64_t x = 0; x < len; ++x) {
        v += (uint32_t)(next(&s) % 4);
        k[x] = v;
    }
}

int main(void) {
    const uint64_t m = 1000003, n = 777777, N = m + n;
    uint32_t *A = malloc(m * 4), *Av = malloc(m * 4), *B = malloc(n * 4), *Bv = malloc(n * 4);
    uint32_t *C = malloc(N * 4), *Cv = malloc(N * 4), *Cr = malloc(N * 4), *Cvr = malloc(N * 4);
    if (!A || !Av || !B || !Bv || !C || !Cv || !Cr || !Cvr) return 2;
    sorted_keys(A, m, 1);
    sorted_keys(B, n, 2);
    for (uint64_t x = 0; x < m; ++x) Av[x] = (uint32_t)x;
    for (uint64_t y = 0; y < n; ++y) Bv[y] = (uint32_t)((1ull << 31) + y);

    void *dA, *dAv, *dB, *dBv, *dC, *dCv, *ws, *dranks, *dj;
    const size_t ws_bytes = cm_merge_workspace_size(CM_KEY_U32, 1, m, n);
    HIP_OK(hipMalloc(&dA, m * 4));
    HIP_OK(hipMalloc(&dAv, m * 4));
    HIP_OK(hipMalloc(&dB, n * 4));
    HIP_OK(hipMalloc(&dBv, n * 4));
    HIP_OK(hipMalloc(&dC, N * 4));
    HIP_OK(hipMalloc(&dCv, N * 4));
    HIP_OK(hipMalloc(&ws, ws_bytes));
    HIP_OK(hipMalloc(&dranks, 5 * 8));
    HIP_OK(hipMalloc(&dj, 5 * 8));
    HIP_OK(hipMemcpy(dA, A, m * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dAv, Av, m * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dB, B, n * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dBv, Bv, n * 4, hipMemcpyHostToDevice));
    hipStream_t st;
    HIP_OK(hipStreamCreate(&st));

    int rc = cm_stable_merge_pairs(CM_KEY_U32, dA, dAv, m, dB, dBv, n, dC, dCv, ws, ws_bytes, st);
    if (rc != CM_OK) {
        fprintf(stderr, "cm_stable_merge_pairs: %s\n", cm_status_string(rc));
        return 1;
    }
    /* argument errors come back before anything is enqueued */
    if (cm_stable_merge_pairs(CM_KEY_U32, dA, dAv, m, dB, dBv, n, dA, dCv, ws, ws_bytes, st) != CM_EALIAS ||
        cm_stable_merge_pairs(CM_KEY_U32, dA, dAv, m, dB, dBv, n, dC, dCv, ws, 8, st) != CM_ENOSPC) {
        fprintf(stderr, "argument errors not reported\n");
        return 1;
    }
    const uint64_t ranks[5] = {0, 1, 123457, N / 2, N};
    HIP_OK(hipMemcpyAsync(dranks, ranks, sizeof ranks, hipMemcpyHostToDevice, st));
    rc = cm_co_rank(CM_KEY_U32, dranks, 5, dA, m, dB, n, dj, st);
    if (rc != CM_OK) {
        fprintf(stderr, "cm_co_rank: %s\n", cm_status_string(rc));
        return 1;
    }
    uint64_t j_dev[5];
    HIP_OK(hipMemcpyAsync(j_dev, dj, sizeof j_dev, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(C, dC, N * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(Cv, dCv, N * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));

    oracle_stable_merge(ORACLE_U32, A, Av, m, B, Bv, n, Cr, Cvr);
    if (memcmp(C, Cr, N * 4) || memcmp(Cv, Cvr, N * 4)) {
        fprintf(stderr, "merge differs from the oracle\n");
        return 1;
    }
    for (int r = 0; r < 5; ++r) {
        uint64_t jh = 0, kh = 0;
        const uint64_t jb = oracle_co_rank_brute(ORACLE_U32, ranks[r], A, m, B, n);
        if (cm_co_rank_host(CM_KEY_U32, ranks[r], A, m, B, n, &jh, &kh) != CM_OK || jh != jb ||
            jh + kh != ranks[r] || j_dev[r] != jb) {
            fprintf(stderr, "co-rank of %llu differs\n", (unsigned long long)ranks[r]);
            return 1;
        }
    }
    /* 8-byte payloads: origin in the high word, side tag in the low word;
       expected from the oracle's origin codes */
    uint64_t *Av64 = malloc(m * 8), *Bv64 = malloc(n * 8), *Cv64 = malloc(N * 8);
    void *dAv64, *dBv64, *dCv64;
    if (!Av64 || !Bv64 || !Cv64) return 2;
    for (uint64_t x = 0; x < m; ++x) Av64[x] = (x << 32) | 0xAu;
    for (uint64_t y = 0; y < n; ++y) Bv64[y] = (y << 32) | 0xBu;
    HIP_OK(hipMalloc(&dAv64, m * 8));
    HIP_OK(hipMalloc(&dBv64, n * 8));
    HIP_OK(hipMalloc(&dCv64, N * 8));
    HIP_OK(hipMemcpy(dAv64, Av64, m * 8, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dBv64, Bv64, n * 8, hipMemcpyHostToDevice));
    rc = cm_stable_merge_pairs64(CM_KEY_U32, dA, dAv64, m, dB, dBv64, n, dC, dCv64, ws, ws_bytes, st);
    if (rc != CM_OK) {
        fprintf(stderr, "cm_stable_merge_pairs64: %s\n", cm_status_string(rc));
        return 1;
    }
    HIP_OK(hipMemcpyAsync(C, dC, N * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(Cv64, dCv64, N * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (memcmp(C, Cr, N * 4)) {
        fprintf(stderr, "8-byte payload merge: keys differ from the oracle\n");
        return 1;
    }
    for (uint64_t i = 0; i < N; ++i) {
        const uint64_t c = Cvr[i];
        const uint64_t want = c < (1u << 31) ? (c << 32) | 0xAu : ((c & 0x7fffffffu) << 32) | 0xBu;
        if (Cv64[i] != want) {
            fprintf(stderr, "8-byte payload of output %llu differs\n", (unsigned long long)i);
            return 1;
        }
    }
    HIP_OK(hipStreamDestroy(st));
    hipFree(dA); hipFree(dAv); hipFree(dB); hipFree(dBv); hipFree(dC); hipFree(dCv);
    hipFree(ws); hipFree(dranks); hipFree(dj); hipFree(dAv64); hipFree(dBv64); hipFree(dCv64);
    printf("c client ok: %llu pairs merged bit-exact (4- and 8-byte payloads), 5 co-ranks\n",
           (unsigned long long)N);
    return 0;
}
