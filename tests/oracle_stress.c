/*
 * Test driver of the C oracle -- TEST INFRASTRUCTURE. Built by
 * tests/test_oracle_robust.py with AddressSanitizer + UndefinedBehaviorSanitizer
 * and, separately, with ThreadSanitizer, together with oracle/fbpq_oracle.c.
 *
 * It builds a seeded random index (xorshift generator, no library RNG) with
 * uneven cell sizes and many empty cells, then runs the multithreaded search
 * and checks that every thread count gives the single-thread result bit for
 * bit. Usage: oracle_stress T N nq L threads
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_search(int D, int T, int M, int Kc, int64_t N, const float *C1, const float *C2,
               const float *R, const int64_t *offsets, const uint8_t *codes, const uint32_t *ids,
               const float *Q, int64_t nq, const int64_t *L, const int32_t *k, int32_t kmax,
               int64_t *out_ids, double *out_d, int64_t *out_ncand, int64_t *out_ncells,
               int nthreads);

static uint64_t g_s = 0x9e3779b97f4a7c15ull;
static uint64_t rnd(void)
{
    g_s ^= g_s << 13;
    g_s ^= g_s >> 7;
    g_s ^= g_s << 17;
    return g_s;
}
static float rndf(float scale) { return (float)((rnd() >> 40) * (1.0 / 16777216.0)) * scale; }

int main(int argc, char **argv)
{
    if (argc != 6) {
        fprintf(stderr, "usage: %s T N nq L threads\n", argv[0]);
        return 2;
    }
    const int T = atoi(argv[1]), D = 32, M = 8, Kc = 256;
    const int64_t N = atoll(argv[2]), nq = atoll(argv[3]), L = atoll(argv[4]);
    const int nth = atoi(argv[5]);
    const int h = D / 2, ds = D / M;
    const int64_t C = (int64_t)T * T;
    float *C1 = malloc(sizeof(float) * T * h), *C2 = malloc(sizeof(float) * T * h);
    float *R = malloc(sizeof(float) * M * Kc * ds), *Q = malloc(sizeof(float) * nq * D);
    int64_t *off = calloc((size_t)C + 1, sizeof(int64_t));
    uint8_t *codes = malloc((size_t)N * M);
    uint32_t *ids = malloc(sizeof(uint32_t) * (size_t)N);
    int64_t *Ls = malloc(sizeof(int64_t) * nq);
    int32_t *ks = malloc(sizeof(int32_t) * nq);
    const int kmax = 16;
    int64_t *id1 = malloc(sizeof(int64_t) * nq * kmax), *idn = malloc(sizeof(int64_t) * nq * kmax);
    double *d1 = malloc(sizeof(double) * nq * kmax), *dn = malloc(sizeof(double) * nq * kmax);
    int64_t *nc1 = malloc(sizeof(int64_t) * nq), *ncn = malloc(sizeof(int64_t) * nq);
    int64_t *nl1 = malloc(sizeof(int64_t) * nq), *nln = malloc(sizeof(int64_t) * nq);
    if (!C1 || !C2 || !R || !Q || !off || !codes || !ids || !Ls || !ks || !id1 || !idn || !d1 || !dn ||
        !nc1 || !ncn || !nl1 || !nln) {
        fprintf(stderr, "allocation failed\n");
        return 2;
    }
    for (int64_t i = 0; i < (int64_t)T * h; ++i) {
        C1[i] = rndf(64.f);
        C2[i] = rndf(64.f);
    }
    for (int64_t i = 0; i < (int64_t)M * Kc * ds; ++i) R[i] = rndf(8.f) - 4.f;
    for (int64_t i = 0; i < nq * D; ++i) Q[i] = rndf(64.f);
    /* points fall in a quarter of the cells, with a skew toward low cell ids */
    for (int64_t p = 0; p < N; ++p) {
        const uint64_t r = rnd();
        const int64_t c = (int64_t)((r % (uint64_t)(C / 4 + 1)) * ((r >> 62) + 1)) % C;
        off[c + 1] += 1;
    }
    for (int64_t c = 0; c < C; ++c) off[c + 1] += off[c];
    for (int64_t p = 0; p < N * M; ++p) codes[p] = (uint8_t)(rnd() >> 56);
    for (int64_t p = 0; p < N; ++p) ids[p] = (uint32_t)(N - 1 - p);
    for (int64_t q = 0; q < nq; ++q) {
        Ls[q] = 1 + (int64_t)(rnd() % (uint64_t)L);
        ks[q] = 1 + (int32_t)(rnd() % kmax);
    }
    if (orc_search(D, T, M, Kc, N, C1, C2, R, off, codes, ids, Q, nq, Ls, ks, kmax, id1, d1, nl1, nc1, 1)) {
        fprintf(stderr, "single-thread search failed\n");
        return 1;
    }
    if (orc_search(D, T, M, Kc, N, C1, C2, R, off, codes, ids, Q, nq, Ls, ks, kmax, idn, dn, nln, ncn, nth)) {
        fprintf(stderr, "%d-thread search failed\n", nth);
        return 1;
    }
    if (memcmp(id1, idn, sizeof(int64_t) * nq * kmax) || memcmp(d1, dn, sizeof(double) * nq * kmax) ||
        memcmp(nl1, nln, sizeof(int64_t) * nq) || memcmp(nc1, ncn, sizeof(int64_t) * nq)) {
        fprintf(stderr, "results differ between 1 and %d threads\n", nth);
        return 1;
    }
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t want = Ls[q] < N ? Ls[q] : N;
        if (nl1[q] != want) {
            fprintf(stderr, "query %lld: %lld candidates, want %lld\n", (long long)q, (long long)nl1[q],
                    (long long)want);
            return 1;
        }
        for (int r = 1; r < ks[q] && r < want; ++r)
            if (d1[q * kmax + r] < d1[q * kmax + r - 1]) {
                fprintf(stderr, "query %lld: distances not ascending\n", (long long)q);
                return 1;
            }
    }
    printf("oracle_stress ok: T=%d N=%lld nq=%lld threads=%d\n", T, (long long)N, (long long)nq, nth);
    free(C1); free(C2); free(R); free(Q); free(off); free(codes); free(ids); free(Ls); free(ks);
    free(id1); free(idn); free(d1); free(dn); free(nc1); free(ncn); free(nl1); free(nln);
    return 0;
}
