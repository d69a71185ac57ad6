/*
 * Test infrastructure: drives every routine of the CPU oracle on small inputs
 * so that tests/test_oracle_sanitize.py can run it under AddressSanitizer and
 * UndefinedBehaviorSanitizer (one translation unit with the oracle source).
 * Prints a few sums; exits non-zero if a routine reports an error.
 */
#include "../oracle/gcmc_oracle.c"

#include <stdio.h>

static double frand(uint64_t* s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static void fill(double* v, int64_t n, double L, uint64_t* s)
{
    for (int64_t i = 0; i < n; ++i)
        v[i] = L * frand(s);
}

int main(void)
{
    const int64_t n = 60, max_n = 400, moves = 500;
    uint64_t st = 20260101;
    oracle_params p;
    memset(&p, 0, sizeof p);
    p.L[0] = 6.5; p.L[1] = 7.0; p.L[2] = 8.0;
    p.rc = 2.5;
    p.ns = 1;
    p.eps[0] = 1.0;
    p.sigma[0] = 1.0;
    p.beta = 1.0 / 1.2;
    p.mu = -3.0;
    p.lambda3 = 1.0;
    p.max_disp = 0.3;
    p.p_disp = 1.0 / 3.0;
    double* x = calloc(max_n, sizeof(double));
    double* y = calloc(max_n, sizeof(double));
    double* z = calloc(max_n, sizeof(double));
    double* e = calloc(max_n, sizeof(double));
    int32_t* sp = calloc(max_n, sizeof(int32_t));
    int64_t* ids = calloc(max_n, sizeof(int64_t));
    oracle_log* lg = calloc(moves, sizeof(oracle_log));
    if (!x || !y || !z || !e || !sp || !ids || !lg)
        return 2;
    fill(x, n, p.L[0], &st);
    fill(y, n, p.L[1], &st);
    fill(z, n, p.L[2], &st);

    double tot[3], pe[2], u[8];
    oracle_total_energy(n, x, y, z, NULL, &p, tot, e);
    oracle_position_energy(n, x, y, z, NULL, 1.0, 2.0, 3.0, 0, -1, &p, pe);
    oracle_move_draws(7, 3, 1, u);
    /* picks at the extremes of both uniforms and of n (one field per pick at 2^31 - 1) */
    const int64_t pn[6] = {1, 2, 3, 37, 1500000, 2147483647};
    const double pu[3] = {0.0, u[7], 1.0 - 1.0 / 9007199254740992.0};
    int64_t picks = 0;
    for (int q = 0; q < 6; ++q)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                int64_t i = oracle_pick(pu[a], pu[b], pn[q]);
                if (i < 0 || i >= pn[q])
                    return 3;
                picks += i;
            }
    int64_t counts[ORACLE_MAX_SPECIES] = {n, 0, 0, 0};
    double tail = oracle_tail_energy(counts, &p) + oracle_tail_delta(counts, 0, +1, &p) +
                  oracle_tail_pressure(counts, &p);
    double arg = oracle_accept_arg(1, 0.5, n, &p);
    int32_t acc = oracle_accept(arg, 0.5, u[3]);

    /* neighbour sets on the paper's grid and on a pruned microcell grid */
    const int32_t req0[3] = {0, 0, 0}, req1[3] = {8, 9, 11};
    int64_t nn0 = oracle_neighbor_ids(n, x, y, z, x[0], y[0], z[0], 0, p.L, p.rc, req0, ids, max_n);
    int64_t nn1 = oracle_neighbor_ids(n, x, y, z, x[1], y[1], z[1], 1, p.L, p.rc, req1, ids, max_n);
    int32_t kept = oracle_stencil_count(p.L, p.rc, req1);
    int32_t M[3], k[3], span[3];
    double invS[3];
    oracle_grid(p.L, p.rc, req1, M, invS, k, span);
    int64_t c = oracle_cell_of(x[2], y[2], z[2], M, invS);

    /* the chain (single species), then gradients and virial of a two-species mixture */
    int64_t nc = n;
    double U = tot[0] + tot[2], Wr = 0.0, pv[2];
    oracle_position_virial(n, x, y, z, NULL, x[0], y[0], z[0], 0, 0, &p, pv);
    int rc = oracle_chain(max_n, x, y, z, &nc, &U, &Wr, &p, 99, 0, 0, moves, lg);
    if (rc != 0)
        return 3;
    /* the CPU-baseline variants of the chain: several threads, a cell list */
    int64_t nc2 = nc;
    double U2 = U, W2 = Wr;
    if (oracle_chain_mt(max_n, x, y, z, &nc2, &U2, &W2, &p, 99, 0, moves, moves, lg, 3) != 0)
        return 3;
    if (oracle_chain_cells(max_n, x, y, z, &nc2, &U2, &W2, &p, 99, 0, 2 * moves, moves, lg) != 0)
        return 3;
    nc = nc2;
    p.ns = 2;
    p.eps[0] = 1.0; p.eps[1] = 0.9; p.eps[2] = 0.9; p.eps[3] = 0.8;
    p.sigma[0] = 1.0; p.sigma[1] = 1.1; p.sigma[2] = 1.1; p.sigma[3] = 1.2;
    for (int64_t i = 0; i < nc; ++i)
        sp[i] = (int32_t)(i & 1);
    double* gx = calloc(nc, sizeof(double));
    double* gy = calloc(nc, sizeof(double));
    double* gz = calloc(nc, sizeof(double));
    double de[ORACLE_MAX_SPECIES * ORACLE_MAX_SPECIES], ds[ORACLE_MAX_SPECIES * ORACLE_MAX_SPECIES], vir[4], g1[3];
    if (!gx || !gy || !gz)
        return 2;
    oracle_gradients(nc, x, y, z, sp, &p, gx, gy, gz, de, ds);
    oracle_particle_gradient(nc, x, y, z, sp, 0, &p, g1);
    oracle_virial(nc, x, y, z, sp, &p, vir);
    oracle_total_energy(nc, x, y, z, sp, &p, tot, NULL);

    printf("n=%lld U=%.6f tail=%.6f acc=%d nn=%lld/%lld kept=%d cell=%lld g=%.6f W=%.6f picks=%lld\n", (long long)nc,
           tot[0], tail, (int)acc, (long long)nn0, (long long)nn1, (int)kept, (long long)c, gx[0] + g1[0], vir[0],
           (long long)picks);
    free(x); free(y); free(z); free(e); free(sp); free(ids); free(lg); free(gx); free(gy); free(gz);
    return 0;
}
