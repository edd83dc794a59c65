/* Driver for the oracle under AddressSanitizer/UndefinedBehaviorSanitizer and
 * ThreadSanitizer (tests/test_oracle_sanitized.py builds it with the oracle's
 * source): every instance kind, both schedules, phased, synchronous and damped
 * updates, the per-level records and replay, on small instances with several
 * worker threads.  Prints OK when every call returned success. */
#include "../oracle/mars_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static double unit(uint64_t seed, uint64_t i) { return (double)(orc_splitmix64(seed, i) >> 11) * 0x1p-53; }

static int run(const orc_instance *in, orc_schedule sc, const char *label)
{
    const int R = 6, cap = 64, N = in->N;
    double *m = calloc((size_t)N * R, sizeof(double)), *E = calloc(R, sizeof(double));
    double *T0 = calloc(R, sizeof(double)), *lastT = calloc(R, sizeof(double));
    double *dpl = calloc((size_t)R * cap, sizeof(double));
    int8_t *s = calloc((size_t)N * R, 1);
    int64_t *sw = calloc(R, sizeof(int64_t)), *lv = calloc(R, sizeof(int64_t)), *caps = calloc(R, sizeof(int64_t));
    int32_t *spl = calloc((size_t)R * cap, sizeof(int32_t)), *own = calloc((size_t)R * cap, sizeof(int32_t));
    int rc = orc_solve_levels(in, &sc, 7, 0, R, NULL, NULL, m, s, E, T0, sw, lv, caps, lastT, 3, NULL, spl, own, dpl,
                              cap);
    /* replay the recorded sweep counts */
    if (!rc)
        rc = orc_solve_levels(in, &sc, 7, 0, R, NULL, NULL, m, s, E, T0, sw, lv, caps, lastT, 2, spl, NULL, NULL, NULL,
                              cap);
    int64_t hits = 0;
    if (!rc && orc_best(E, R, &hits) < 0)
        rc = 1;
    if (!rc) {
        const double e = orc_energy(in, s);
        (void)e;
    }
    printf("%s: rc %d, best hits %lld\n", label, rc, (long long)hits);
    free(m), free(E), free(T0), free(lastT), free(dpl), free(s), free(sw), free(lv), free(caps), free(spl), free(own);
    return rc;
}

int main(void)
{
    int fails = 0;
    /* dense SK-like, N = 37 (ragged phases), with a field */
    const int Nd = 37;
    float *J = calloc((size_t)Nd * Nd, sizeof(float)), *h = calloc(Nd, sizeof(float));
    for (int i = 0; i < Nd; ++i) {
        h[i] = (float)(unit(3, 100000 + i) - 0.5);
        for (int j = i + 1; j < Nd; ++j)
            J[(size_t)i * Nd + j] = J[(size_t)j * Nd + i] = (float)(unit(1, (uint64_t)i * Nd + j) - 0.5);
    }
    orc_instance dense = {ORC_DENSE, Nd, J, NULL, NULL, NULL, 0, {0, 0, 0}, NULL, h};
    orc_schedule geo = {ORC_GEOMETRIC, 0.5, 3.0, 0.05, 1.0, 12, 1, 1e-4, ORC_PHASED, 3, 1.0, 0, -1};
    orc_schedule paper = {ORC_LINEAR, 0.0, 2.0, 0.0, 0.25, 0, 40, 1e-4, ORC_PHASED, 4, 1.0, 0, -1};
    fails += run(&dense, geo, "dense geometric") != 0;
    fails += run(&dense, paper, "dense paper schedule") != 0;
    orc_schedule damped = geo;
    damped.damping = 0.5;
    damped.update = ORC_JACOBI;
    fails += run(&dense, damped, "dense damped synchronous") != 0;
    /* CSR ring plus chords, int8 weights */
    const int Nc = 29;
    int32_t *rp = calloc(Nc + 1, sizeof(int32_t)), *col = calloc(4 * Nc, sizeof(int32_t));
    int8_t *val = calloc(4 * Nc, 1);
    int nnz = 0;
    for (int i = 0; i < Nc; ++i) {
        rp[i] = nnz;
        const int nb[4] = {(i + 1) % Nc, (i + Nc - 1) % Nc, (i + 7) % Nc, (i + Nc - 7) % Nc};
        for (int k = 0; k < 4; ++k) {
            col[nnz] = nb[k];
            const int a = i < nb[k] ? i : nb[k], b = i < nb[k] ? nb[k] : i;
            val[nnz] = (int8_t)((int)(unit(5, (uint64_t)a * Nc + b) * 200.0) - 100);
            ++nnz;
        }
    }
    rp[Nc] = nnz;
    orc_instance csr = {ORC_CSR, Nc, NULL, rp, col, val, 0, {0, 0, 0}, NULL, NULL};
    fails += run(&csr, geo, "csr geometric") != 0;
    fails += run(&csr, paper, "csr paper schedule") != 0;
    /* 3D lattice 4 x 3 x 5 with +-1 bonds and a field */
    const int L0 = 4, L1 = 3, L2 = 5, Nl = L0 * L1 * L2;
    int8_t *bond = calloc(3 * (size_t)Nl, 1);
    float *hl = calloc(Nl, sizeof(float));
    for (int i = 0; i < 3 * Nl; ++i)
        bond[i] = unit(9, i) < 0.5 ? -1 : 1;
    for (int i = 0; i < Nl; ++i)
        hl[i] = (float)(unit(11, i) - 0.5);
    orc_instance lat = {ORC_LATTICE, Nl, NULL, NULL, NULL, NULL, 3, {L0, L1, L2}, bond, hl};
    fails += run(&lat, geo, "lattice geometric") != 0;
    fails += run(&lat, damped, "lattice damped synchronous") != 0;
    free(J), free(h), free(rp), free(col), free(val), free(bond), free(hl);
    if (fails) {
        printf("FAILED %d\n", fails);
        return 1;
    }
    printf("OK\n");
    return 0;
}
