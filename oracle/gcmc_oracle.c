/*
 * gcmc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU reference for the grand-canonical
 * Monte Carlo (GCMC) energy path of Schwiebert et al., "An Efficient Cell List
 * Implementation for Monte Carlo Simulation on GPUs" (arXiv 1408.3764).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code, header, table or constant with the GPU
 * library; the two are written independently from the paper and from the
 * readings listed in the project's design notes.
 *
 * Every energy here is the plain all-pairs definition (the cell list of the
 * paper only prunes pairs beyond the cutoff, so its result is the all-pairs
 * result).  The one cell-list routine in this file exists only to check the
 * GPU's cell assignment and neighbour sets bit-exactly.
 *
 * Compile with -O2 -ffp-contract=off (no FMA contraction anywhere).
 *
 * Pins (tests that tie this file to the paper and to mathematics rather than
 * to itself) cover: the pair potential (closed forms), the tail correction
 * (numerical quadrature and exact rational differences), minimum image (two-
 * particle box across the boundary), half-sum identity, translation
 * invariance, cell list = all-pairs brute force, the paper's worked numbers
 * for the cell grid, the ideal-gas Poisson limit of the acceptance rules,
 * Philox known-answer vectors, and finite differences for the gradients.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_SPECIES 4

/* Force field, box and ensemble parameters.  eps/sigma are pair tables
 * (ns x ns, symmetric), already mixed by the caller. */
typedef struct {
    double L[3];
    double rc;
    int32_t ns;
    int32_t pad0;
    double eps[ORACLE_MAX_SPECIES * ORACLE_MAX_SPECIES];
    double sigma[ORACLE_MAX_SPECIES * ORACLE_MAX_SPECIES];
    double beta;      /* 1/(k_B T), Eq. (2) */
    double mu;        /* chemical potential, Eqs. (4)-(5) */
    double lambda3;   /* thermal de Broglie wavelength cubed, Eqs. (4)-(5) */
    double max_disp;  /* half-width of the uniform displacement cube */
    double p_disp;    /* DisplacePercent of Algorithm 1 (as a fraction) */
} oracle_params;

/* One record per attempted move of the chain. */
typedef struct {
    int32_t type;      /* 0 displacement, 1 insertion, 2 deletion */
    int32_t index;     /* particle index (displacement/deletion), new id (insertion) */
    int32_t accepted;  /* 1 if the move was accepted */
    int32_t flags;     /* bit0: rejected because N == 0 */
    double dU_pair;    /* pair part of the energy change */
    double dU_tail;    /* tail-correction part of the energy change */
    double sumabs;     /* sum of |u| over the terms of dU_pair (tolerance scale) */
    double x, y, z;    /* trial position (new position / insertion point / deleted particle) */
    double arg;        /* log of the acceptance ratio */
    double a;          /* the uniform A of the acceptance test */
    double dW_pair;    /* change of the pair virial W the move would make */
    double wsumabs;    /* sum of |w| over the terms of dW_pair (tolerance scale) */
} oracle_log;

/* ------------------------------------------------------------------------ */
/* Compensated summation (Neumaier's variant of Kahan summation).           */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, written from its definition in    */
/* Salmon, Moraes, Dror and Shaw, "Parallel Random Numbers: As Easy as      */
/* 1, 2, 3", SC'11: ten rounds, each a pair of 32x32->64 multiplications    */
/* by the two round multipliers, with the key bumped by the two Weyl        */
/* constants between rounds.                                                */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A double in [0,1) from two 32-bit words: 27 high bits of a, 26 of b. */
double oracle_u01(uint32_t a, uint32_t b)
{
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

/* The eight uniforms of one move.  key = (seed low, seed high);
 * counter = (move low, move high, box id, j) for j = 0..3; each call gives
 * two doubles, from output words (0,1) and (2,3).
 *   u[0] = R of Algorithm 1 (move type)     u[1] = Source of Algorithm 1
 *   u[2] = particle pick                    u[3] = A of the acceptance test
 *   u[4..6] = position / displacement       u[7] = pick fields (oracle_pick) */
void oracle_move_draws(uint64_t seed, uint64_t move, uint32_t box, double u[8])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t j = 0; j < 4; ++j) {
        uint32_t ctr[4] = {(uint32_t)move, (uint32_t)(move >> 32), box, j};
        uint32_t w[4];
        oracle_philox4x32_10(ctr, key, w);
        u[2 * j] = oracle_u01(w[0], w[1]);
        u[2 * j + 1] = oracle_u01(w[2], w[3]);
    }
}

/* The random particle of a displacement (Algorithm 2) or a deletion        */
/* (Algorithm 5) among n >= 1 particles.  The paper asks only for a uniform */
/* pick; this one is uniform and rarely changes when n changes by a few:    */
/* with b the smallest bit count such that 2^b >= n, the 53 bits of u_spare */
/* (u_spare = k / 2^53) are cut into floor(53 / b) fields of b bits, high   */
/* field first; the pick is the first field whose value is below n.  When   */
/* none is, it is min(floor(u_pick n), n - 1).  Each field is uniform on    */
/* 0 .. 2^b - 1 and independent of the others and of u_pick, so every index */
/* has probability 1/n.                                                     */
int64_t oracle_pick(double u_pick, double u_spare, int64_t n)
{
    int b = 0;
    while (((int64_t)1 << b) < n)
        b++;
    if (b == 0)
        return 0;
    uint64_t k = (uint64_t)(u_spare * 9007199254740992.0);
    int fields = 53 / b;
    for (int t = 1; t <= fields; ++t) {
        uint64_t v = (k >> (53 - b * t)) & (((uint64_t)1 << b) - 1);
        if (v < (uint64_t)n)
            return (int64_t)v;
    }
    int64_t i = (int64_t)floor(u_pick * (double)n);
    if (i > n - 1)
        i = n - 1;
    return i;
}

/* ------------------------------------------------------------------------ */
/* Lennard-Jones pair energy, Eq. (1), truncated (not shifted) at rc: only  */
/* pairs strictly inside the cutoff contribute (Sec. 1 and Algorithm 3).    */
/* ------------------------------------------------------------------------ */
double oracle_lj_r2(double r2, double eps, double sigma, double rc)
{
    if (!(r2 < rc * rc))
        return 0.0;
    if (eps == 0.0)
        return 0.0;
    if (r2 == 0.0)
        return INFINITY;
    double sr2 = (sigma * sigma) / r2;
    double sr6 = sr2 * sr2 * sr2;
    double sr12 = sr6 * sr6;
    return 4.0 * eps * (sr12 - sr6);
}

/* Minimum-image separation along one axis of length L (coordinates are kept
 * in [0, L)).  This is the "true distance under periodic boundary
 * conditions" of Algorithms 3, 4, 6 and 7. */
double oracle_min_image(double d, double L)
{
    double h = 0.5 * L;
    if (d > h)
        d -= L;
    else if (d < -h)
        d += L;
    return d;
}

double oracle_dist2(const double L[3], double xi, double yi, double zi, double xj, double yj, double zj)
{
    double dx = oracle_min_image(xj - xi, L[0]);
    double dy = oracle_min_image(yj - yi, L[1]);
    double dz = oracle_min_image(zj - zi, L[2]);
    return (dx * dx + dy * dy) + dz * dz;
}

static double pair_u(const oracle_params* p, int32_t a, int32_t b, double r2)
{
    int ns = p->ns;
    return oracle_lj_r2(r2, p->eps[a * ns + b], p->sigma[a * ns + b], p->rc);
}

/* Energy of a particle of species ps at (px,py,pz) with every particle j of
 * the configuration except `exclude` (Algorithms 3 and 4: one contribution
 * per other particle).  sumabs = sum of |u| (scale for tolerances). */
void oracle_position_energy(int64_t n, const double* x, const double* y, const double* z, const int32_t* sp,
                            double px, double py, double pz, int32_t ps, int64_t exclude,
                            const oracle_params* p, double out[2])
{
    nsum s = {0, 0}, a = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == exclude)
            continue;
        double r2 = oracle_dist2(p->L, px, py, pz, x[j], y[j], z[j]);
        double u = pair_u(p, ps, sp ? sp[j] : 0, r2);
        nsum_add(&s, u);
        nsum_add(&a, fabs(u));
    }
    out[0] = nsum_get(&s);
    out[1] = nsum_get(&a);
}

/* Pair virial w = -r du/dr of the truncated potential (Eq. 1 differentiated):
 * 24 eps [2 (sigma/r)^12 - (sigma/r)^6] strictly inside the cutoff, else 0. */
static double pair_w(const oracle_params* p, int32_t a, int32_t b, double r2);

/* Virial of a particle of species ps at (px,py,pz) with every particle j
 * except `exclude`: sum_j w(r_ij), the quantity an accepted move changes in
 * the running pressure (Sec. 3.1.2).  out[1] = sum of |w|. */
void oracle_position_virial(int64_t n, const double* x, const double* y, const double* z, const int32_t* sp,
                            double px, double py, double pz, int32_t ps, int64_t exclude,
                            const oracle_params* p, double out[2])
{
    nsum s = {0, 0}, a = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == exclude)
            continue;
        double r2 = oracle_dist2(p->L, px, py, pz, x[j], y[j], z[j]);
        double w = pair_w(p, ps, sp ? sp[j] : 0, r2);
        nsum_add(&s, w);
        nsum_add(&a, fabs(w));
    }
    out[0] = nsum_get(&s);
    out[1] = nsum_get(&a);
}

/* Total pair energy over the N(N-1)/2 unique pairs (Sec. 3.1.1), and the
 * per-particle energies e_i = sum_{j != i} u(r_ij) when e != NULL.
 * out[0] = U_pair, out[1] = sum over pairs of |u|, out[2] = U_tail. */
double oracle_tail_energy(const int64_t* counts, const oracle_params* p);

void oracle_total_energy(int64_t n, const double* x, const double* y, const double* z, const int32_t* sp,
                         const oracle_params* p, double out[3], double* e)
{
    nsum s = {0, 0}, a = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double r2 = oracle_dist2(p->L, x[i], y[i], z[i], x[j], y[j], z[j]);
            double u = pair_u(p, sp ? sp[i] : 0, sp ? sp[j] : 0, r2);
            nsum_add(&s, u);
            nsum_add(&a, fabs(u));
        }
    }
    out[0] = nsum_get(&s);
    out[1] = nsum_get(&a);
    int64_t counts[ORACLE_MAX_SPECIES] = {0};
    for (int64_t i = 0; i < n; ++i)
        counts[sp ? sp[i] : 0] += 1;
    out[2] = oracle_tail_energy(counts, p);
    if (e) {
        for (int64_t i = 0; i < n; ++i) {
            double pe[2];
            oracle_position_energy(n, x, y, z, sp, x[i], y[i], z[i], sp ? sp[i] : 0, i, p, pe);
            e[i] = pe[0];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Tail correction (Sec. 1 names it; the paper gives no formula).  The      */
/* textbook closed form for a truncated LJ potential with a uniform pair    */
/* distribution beyond rc, ordered double sum over species:                 */
/*   U_tail = (8 pi / (3 V)) sum_a sum_b N_a N_b K_ab,                     */
/*   K_ab = eps_ab sigma_ab^3 [ (sigma_ab/rc)^9 / 3 - (sigma_ab/rc)^3 ].     */
/* ------------------------------------------------------------------------ */
static double tail_k(const oracle_params* p, int a, int b)
{
    int ns = p->ns;
    double eps = p->eps[a * ns + b], sig = p->sigma[a * ns + b];
    double q = sig / p->rc;
    double q3 = q * q * q;
    double q9 = q3 * q3 * q3;
    return eps * sig * sig * sig * (q9 / 3.0 - q3);
}

static double box_volume(const oracle_params* p) { return (p->L[0] * p->L[1]) * p->L[2]; }

double oracle_tail_energy(const int64_t* counts, const oracle_params* p)
{
    double V = box_volume(p);
    double s = 0.0;
    for (int a = 0; a < p->ns; ++a)
        for (int b = 0; b < p->ns; ++b)
            s += (double)counts[a] * (double)counts[b] * tail_k(p, a, b);
    return (8.0 * M_PI / (3.0 * V)) * s;
}

/* U_tail(N + sign * e_s) - U_tail(N), expanded algebraically from the closed
 * form above (sign = +1 insertion, -1 deletion of a particle of species s):
 *   (8 pi/(3V)) [ 2 sign sum_b N_b K_sb + K_ss ]. */
double oracle_tail_delta(const int64_t* counts, int32_t s, int32_t sign, const oracle_params* p)
{
    double V = box_volume(p);
    double acc = 0.0;
    for (int b = 0; b < p->ns; ++b)
        acc += (double)counts[b] * tail_k(p, s, b);
    return (8.0 * M_PI / (3.0 * V)) * (2.0 * (double)sign * acc + tail_k(p, s, s));
}

/* ------------------------------------------------------------------------ */
/* Acceptance, Eqs. (2)-(5).  arg is the log of the ratio inside min[1, .]. */
/*   displacement:  -beta dU                                   (Eq. 3)      */
/*   insertion:     ln(V / (Lambda^3 (N+1))) + beta (mu - dU)  (Eq. 4, with */
/*                  the sign of the exponent read as in Eq. 5 / Frenkel &   */
/*                  Smit)                                                   */
/*   deletion:      ln(Lambda^3 N / V) - beta (mu + dU)        (Eq. 5)      */
/* Accept iff arg >= 0 or A < exp(arg), with A uniform in [0,1); a NaN dU   */
/* is rejected.                                                             */
/* ------------------------------------------------------------------------ */
double oracle_accept_arg(int32_t type, double dU, int64_t n, const oracle_params* p)
{
    double V = box_volume(p);
    if (type == 0)
        return -(p->beta * dU);
    if (type == 1)
        return log(V / (p->lambda3 * (double)(n + 1))) + p->beta * (p->mu - dU);
    return log((p->lambda3 * (double)n) / V) - p->beta * (p->mu + dU);
}

int32_t oracle_accept(double arg, double dU, double A)
{
    if (isnan(dU))
        return 0;
    if (arg >= 0.0)
        return 1;
    return A < exp(arg) ? 1 : 0;
}

/* Periodic wrap of a coordinate back into [0, L). */
static double wrap_coord(double x, double L)
{
    if (x >= L)
        x -= L;
    else if (x < 0.0)
        x += L;
    if (x >= L)
        x = 0.0;
    return x;
}

/* ------------------------------------------------------------------------ */
/* The serial GCMC chain of Algorithm 1, with the displacement of           */
/* Algorithm 2 and the insertion/deletion of Algorithm 5, every energy      */
/* change computed all-pairs.  Single species only.                         */
/*                                                                          */
/* Per move (counter = counter0 + m):                                       */
/*   R < p_disp -> displacement; else Source < 0.5 -> deletion; else        */
/*   insertion.  Displacement and deletion pick i = oracle_pick(u2, u7, N)  */
/*   and are rejected when N == 0.  Displacement: x' = wrap(x + d (2u-1))   */
/*   per axis.  Insertion: x = wrap(L u).  On accepted insertion the new    */
/*   particle gets index N; on accepted deletion particle N-1 takes index i.*/
/* State: x,y,z[max_n], *n, *U (total energy incl. tail, running), *W (pair */
/* virial, running; may be NULL).  Each move's virial change is computed    */
/* like its energy change and applied on acceptance (Sec. 3.1.2).           */
/* Returns 0, or -1 if an insertion would exceed max_n (an error, never a   */
/* rejection), or -2 for an unsupported parameter set.                      */
/* ------------------------------------------------------------------------ */
struct cell_list;
/* How the chain sums a position's pair energy and virial: over all particles
 * (threads == 1: the plain loops of oracle_position_energy/virial; threads >
 * 1: the same terms in `threads` contiguous index ranges summed at once and
 * combined in range order), or over the stencil cells of a cell list. */
typedef struct {
    int threads;
    struct cell_list* cells;
} sum_mode;

static void position_sums(const sum_mode* md, int64_t n, const double* x, const double* y, const double* z,
                          double px, double py, double pz, int64_t exclude, const oracle_params* p, double e[2],
                          double w[2]);
static void cells_insert(struct cell_list* cl, int64_t i, double px, double py, double pz);
static void cells_remove(struct cell_list* cl, int64_t i);
static void cells_relabel(struct cell_list* cl, int64_t from, int64_t to);

static int chain_run(const sum_mode* md, int64_t max_n, double* x, double* y, double* z, int64_t* n_io,
                     double* U_io, double* W_io, const oracle_params* p, uint64_t seed, uint32_t box,
                     uint64_t counter0, int64_t n_moves, oracle_log* log_out)
{
    if (p->ns != 1)
        return -2;
    int64_t n = *n_io;
    double U = *U_io;
    double W = W_io ? *W_io : 0.0;
    for (int64_t m = 0; m < n_moves; ++m) {
        double u[8];
        oracle_move_draws(seed, counter0 + (uint64_t)m, box, u);
        oracle_log rec;
        memset(&rec, 0, sizeof rec);
        int32_t type;
        if (u[0] < p->p_disp)
            type = 0;
        else if (u[1] < 0.5)
            type = 2;
        else
            type = 1;
        rec.type = type;
        rec.a = u[3];
        if (type != 1 && n == 0) {
            rec.index = -1;
            rec.flags = 1;
            rec.accepted = 0;
            if (log_out)
                log_out[m] = rec;
            continue;
        }
        int64_t i = 0;
        if (type != 1)
            i = oracle_pick(u[2], u[7], n);
        double dUp = 0.0, dUt = 0.0, sabs = 0.0, dWp = 0.0, wabs = 0.0;
        double nx = 0, ny = 0, nz = 0;
        if (type == 0) {
            nx = wrap_coord(x[i] + p->max_disp * (2.0 * u[4] - 1.0), p->L[0]);
            ny = wrap_coord(y[i] + p->max_disp * (2.0 * u[5] - 1.0), p->L[1]);
            nz = wrap_coord(z[i] + p->max_disp * (2.0 * u[6] - 1.0), p->L[2]);
            double eo[2], en[2], wo[2], wn[2];
            position_sums(md, n, x, y, z, x[i], y[i], z[i], i, p, eo, wo);
            position_sums(md, n, x, y, z, nx, ny, nz, i, p, en, wn);
            dUp = en[0] - eo[0];
            sabs = en[1] + eo[1];
            dWp = wn[0] - wo[0];
            wabs = wn[1] + wo[1];
            rec.index = (int32_t)i;
        } else if (type == 1) {
            nx = wrap_coord(p->L[0] * u[4], p->L[0]);
            ny = wrap_coord(p->L[1] * u[5], p->L[1]);
            nz = wrap_coord(p->L[2] * u[6], p->L[2]);
            double en[2], wn[2];
            position_sums(md, n, x, y, z, nx, ny, nz, -1, p, en, wn);
            int64_t counts[1] = {n};
            dUp = en[0];
            sabs = en[1];
            dWp = wn[0];
            wabs = wn[1];
            dUt = oracle_tail_delta(counts, 0, +1, p);
            rec.index = (int32_t)n;
        } else {
            nx = x[i]; ny = y[i]; nz = z[i];
            double eo[2], wo[2];
            position_sums(md, n, x, y, z, x[i], y[i], z[i], i, p, eo, wo);
            int64_t counts[1] = {n};
            dUp = -eo[0];
            sabs = eo[1];
            dWp = -wo[0];
            wabs = wo[1];
            dUt = oracle_tail_delta(counts, 0, -1, p);
            rec.index = (int32_t)i;
        }
        double dU = dUp + dUt;
        double arg = oracle_accept_arg(type, dU, n, p);
        int32_t acc = oracle_accept(arg, dU, u[3]);
        rec.dU_pair = dUp;
        rec.dU_tail = dUt;
        rec.sumabs = sabs;
        rec.dW_pair = dWp;
        rec.wsumabs = wabs;
        rec.x = nx; rec.y = ny; rec.z = nz;
        rec.arg = arg;
        if (acc) {
            if (type == 0) {
                if (md->cells)
                    cells_remove(md->cells, i);
                x[i] = nx; y[i] = ny; z[i] = nz;
                if (md->cells)
                    cells_insert(md->cells, i, nx, ny, nz);
            } else if (type == 1) {
                if (n >= max_n) {
                    *n_io = n;
                    *U_io = U;
                    if (W_io)
                        *W_io = W;
                    return -1;
                }
                x[n] = nx; y[n] = ny; z[n] = nz;
                if (md->cells)
                    cells_insert(md->cells, n, nx, ny, nz);
                n += 1;
            } else {
                if (md->cells) {
                    cells_remove(md->cells, i);
                    if (i != n - 1)
                        cells_relabel(md->cells, n - 1, i);
                }
                x[i] = x[n - 1]; y[i] = y[n - 1]; z[i] = z[n - 1];
                n -= 1;
            }
            U += dU;
            W += dWp;
        }
        rec.accepted = acc;
        if (log_out)
            log_out[m] = rec;
    }
    *n_io = n;
    *U_io = U;
    if (W_io)
        *W_io = W;
    return 0;
}

int oracle_chain(int64_t max_n, double* x, double* y, double* z, int64_t* n_io, double* U_io, double* W_io,
                 const oracle_params* p, uint64_t seed, uint32_t box, uint64_t counter0, int64_t n_moves,
                 oracle_log* log_out)
{
    sum_mode md = {1, NULL};
    return chain_run(&md, max_n, x, y, z, n_io, U_io, W_io, p, seed, box, counter0, n_moves, log_out);
}

/* ------------------------------------------------------------------------ */
/* The same chain for the CPU baselines of the measurements (not used by    */
/* the parity tests): all pairs on several threads, and a cell list.        */
/* ------------------------------------------------------------------------ */
#define ORACLE_MAX_THREADS 256

static void range_sums(int64_t j0, int64_t j1, const double* x, const double* y, const double* z, double px,
                       double py, double pz, int64_t exclude, const oracle_params* p, nsum acc[4])
{
    for (int64_t j = j0; j < j1; ++j) {
        if (j == exclude)
            continue;
        double r2 = oracle_dist2(p->L, px, py, pz, x[j], y[j], z[j]);
        double u = pair_u(p, 0, 0, r2);
        double w = pair_w(p, 0, 0, r2);
        nsum_add(&acc[0], u);
        nsum_add(&acc[1], fabs(u));
        nsum_add(&acc[2], w);
        nsum_add(&acc[3], fabs(w));
    }
}

/* The plain cell list of Sec. 3.2 on the host: each cell a doubly linked list
 * of particle indices (O(1) insertion and removal), the paper's grid
 * (M = max(3, floor(L / rc)), stencil of 2k + 1 cells per axis, whole axis
 * when that covers it). */
typedef struct cell_list {
    int32_t M[3], k[3], span[3];
    double invS[3];
    int64_t ncells;
    int64_t* head;
    int64_t* next;
    int64_t* prev;
    int64_t* cell;
} cell_list;

static int32_t axis_cell(double x, double invS, int32_t M);

static void cells_insert(cell_list* cl, int64_t i, double px, double py, double pz)
{
    int64_t c = ((int64_t)axis_cell(pz, cl->invS[2], cl->M[2]) * cl->M[1] + axis_cell(py, cl->invS[1], cl->M[1])) *
                    cl->M[0] + axis_cell(px, cl->invS[0], cl->M[0]);
    cl->cell[i] = c;
    cl->prev[i] = -1;
    cl->next[i] = cl->head[c];
    if (cl->head[c] >= 0)
        cl->prev[cl->head[c]] = i;
    cl->head[c] = i;
}

static void cells_remove(cell_list* cl, int64_t i)
{
    int64_t c = cl->cell[i];
    if (cl->prev[i] >= 0)
        cl->next[cl->prev[i]] = cl->next[i];
    else
        cl->head[c] = cl->next[i];
    if (cl->next[i] >= 0)
        cl->prev[cl->next[i]] = cl->prev[i];
}

/* Particle `from` takes index `to` (which is in no cell). */
static void cells_relabel(cell_list* cl, int64_t from, int64_t to)
{
    int64_t c = cl->cell[from];
    cl->cell[to] = c;
    cl->prev[to] = cl->prev[from];
    cl->next[to] = cl->next[from];
    if (cl->prev[to] >= 0)
        cl->next[cl->prev[to]] = to;
    else
        cl->head[c] = to;
    if (cl->next[to] >= 0)
        cl->prev[cl->next[to]] = to;
}

static void cell_sums(const cell_list* cl, const double* x, const double* y, const double* z, double px,
                      double py, double pz, int64_t exclude, const oracle_params* p, nsum acc[4])
{
    int32_t c0[3] = {axis_cell(px, cl->invS[0], cl->M[0]), axis_cell(py, cl->invS[1], cl->M[1]),
                     axis_cell(pz, cl->invS[2], cl->M[2])};
    int32_t lo[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
        int full = cl->span[a] == cl->M[a];
        lo[a] = full ? 0 : c0[a] - cl->k[a];
        cnt[a] = full ? cl->M[a] : 2 * cl->k[a] + 1;
    }
    for (int32_t tz = 0; tz < cnt[2]; ++tz) {
        int32_t cz = ((lo[2] + tz) % cl->M[2] + cl->M[2]) % cl->M[2];
        for (int32_t ty = 0; ty < cnt[1]; ++ty) {
            int32_t cy = ((lo[1] + ty) % cl->M[1] + cl->M[1]) % cl->M[1];
            for (int32_t tx = 0; tx < cnt[0]; ++tx) {
                int32_t cx = ((lo[0] + tx) % cl->M[0] + cl->M[0]) % cl->M[0];
                for (int64_t j = cl->head[((int64_t)cz * cl->M[1] + cy) * cl->M[0] + cx]; j >= 0; j = cl->next[j]) {
                    if (j == exclude)
                        continue;
                    double r2 = oracle_dist2(p->L, px, py, pz, x[j], y[j], z[j]);
                    double u = pair_u(p, 0, 0, r2);
                    double w = pair_w(p, 0, 0, r2);
                    nsum_add(&acc[0], u);
                    nsum_add(&acc[1], fabs(u));
                    nsum_add(&acc[2], w);
                    nsum_add(&acc[3], fabs(w));
                }
            }
        }
    }
}

static void position_sums(const sum_mode* md, int64_t n, const double* x, const double* y, const double* z,
                          double px, double py, double pz, int64_t exclude, const oracle_params* p, double e[2],
                          double w[2])
{
    if (!md->cells && md->threads <= 1) {
        oracle_position_energy(n, x, y, z, NULL, px, py, pz, 0, exclude, p, e);
        oracle_position_virial(n, x, y, z, NULL, px, py, pz, 0, exclude, p, w);
        return;
    }
    nsum tot[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (md->cells) {
        cell_sums(md->cells, x, y, z, px, py, pz, exclude, p, tot);
    } else {
        int T = md->threads > ORACLE_MAX_THREADS ? ORACLE_MAX_THREADS : md->threads;
        nsum part[ORACLE_MAX_THREADS][4];
#pragma omp parallel for num_threads(T) schedule(static, 1)
        for (int t = 0; t < T; ++t) {
            for (int q = 0; q < 4; ++q)
                part[t][q].s = part[t][q].c = 0.0;
            range_sums(n * t / T, n * (t + 1) / T, x, y, z, px, py, pz, exclude, p, part[t]);
        }
        for (int t = 0; t < T; ++t)
            for (int q = 0; q < 4; ++q) {
                nsum_add(&tot[q], part[t][q].s);
                nsum_add(&tot[q], part[t][q].c);
            }
    }
    e[0] = nsum_get(&tot[0]);
    e[1] = nsum_get(&tot[1]);
    w[0] = nsum_get(&tot[2]);
    w[1] = nsum_get(&tot[3]);
}

/* oracle_chain with every position's sums split over `threads` threads. */
int oracle_chain_mt(int64_t max_n, double* x, double* y, double* z, int64_t* n_io, double* U_io, double* W_io,
                    const oracle_params* p, uint64_t seed, uint32_t box, uint64_t counter0, int64_t n_moves,
                    oracle_log* log_out, int32_t threads)
{
    sum_mode md = {threads < 1 ? 1 : threads, NULL};
    return chain_run(&md, max_n, x, y, z, n_io, U_io, W_io, p, seed, box, counter0, n_moves, log_out);
}

void oracle_grid(const double L[3], double rc, const int32_t req_m[3], int32_t M[3], double invS[3],
                 int32_t k[3], int32_t span[3]);

/* oracle_chain with every position's sums taken over its stencil cells (the
 * paper's grid), the cell list kept current move by move (Sec. 3.2.5).
 * Returns -3 if the cell list cannot be allocated. */
int oracle_chain_cells(int64_t max_n, double* x, double* y, double* z, int64_t* n_io, double* U_io, double* W_io,
                       const oracle_params* p, uint64_t seed, uint32_t box, uint64_t counter0, int64_t n_moves,
                       oracle_log* log_out)
{
    cell_list cl;
    memset(&cl, 0, sizeof cl);
    oracle_grid(p->L, p->rc, NULL, cl.M, cl.invS, cl.k, cl.span);
    cl.ncells = (int64_t)cl.M[0] * cl.M[1] * cl.M[2];
    cl.head = malloc(sizeof(int64_t) * (size_t)cl.ncells);
    cl.next = malloc(sizeof(int64_t) * (size_t)(max_n > 0 ? max_n : 1));
    cl.prev = malloc(sizeof(int64_t) * (size_t)(max_n > 0 ? max_n : 1));
    cl.cell = malloc(sizeof(int64_t) * (size_t)(max_n > 0 ? max_n : 1));
    int rc = -3;
    if (cl.head && cl.next && cl.prev && cl.cell) {
        for (int64_t c = 0; c < cl.ncells; ++c)
            cl.head[c] = -1;
        for (int64_t i = *n_io - 1; i >= 0; --i)
            cells_insert(&cl, i, x[i], y[i], z[i]);
        sum_mode md = {1, &cl};
        rc = chain_run(&md, max_n, x, y, z, n_io, U_io, W_io, p, seed, box, counter0, n_moves, log_out);
    }
    free(cl.head);
    free(cl.next);
    free(cl.prev);
    free(cl.cell);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Cell grid and neighbour sets, used only to check the GPU's cell list     */
/* bit-exactly (Sec. 3.2).                                                  */
/*                                                                          */
/* Cells per axis: the largest T with S = L/T >= rc, at least 3 (the paper's*/
/* rule: "if L < 3 rc, S = L/3"), i.e. M = max(3, floor(L/rc)); a request   */
/* req_m > 0 overrides it (smaller cells).  invS = M/L.  Half-width of the  */
/* stencil k = ceil(rc invS); the stencil along an axis is the 2k+1 cells   */
/* around the particle's cell with periodic wrap, or all M cells when       */
/* 2k+1 >= M.  Cell of a coordinate: min(floor(x invS), M-1).               */
/* ------------------------------------------------------------------------ */
void oracle_grid(const double L[3], double rc, const int32_t req_m[3], int32_t M[3], double invS[3],
                 int32_t k[3], int32_t span[3])
{
    for (int a = 0; a < 3; ++a) {
        int32_t m = (int32_t)floor(L[a] / rc);
        if (m < 3)
            m = 3;
        if (req_m && req_m[a] > 0)
            m = req_m[a];
        M[a] = m;
        invS[a] = (double)m / L[a];
        int32_t kk = (int32_t)ceil(rc * invS[a]);
        if (kk < 1)
            kk = 1;
        k[a] = kk;
        span[a] = (2 * kk + 1 >= m) ? m : 2 * kk + 1;
    }
}

static int32_t axis_cell(double x, double invS, int32_t M)
{
    int64_t c = (int64_t)floor(x * invS);
    if (c > M - 1)
        c = M - 1;
    if (c < 0)
        c = 0;
    return (int32_t)c;
}

int64_t oracle_cell_of(double x, double y, double z, const int32_t M[3], const double invS[3])
{
    int64_t cx = axis_cell(x, invS[0], M[0]);
    int64_t cy = axis_cell(y, invS[1], M[1]);
    int64_t cz = axis_cell(z, invS[2], M[2]);
    return (cz * M[1] + cy) * M[0] + cx;
}

/* Axis-wise stencil membership: is cell coordinate c within the stencil of
 * centre coordinate c0 on an axis of M cells with half-width k? */
static int in_axis_stencil(int32_t c, int32_t c0, int32_t k, int32_t M)
{
    if (2 * k + 1 >= M)
        return 1;
    for (int32_t t = -k; t <= k; ++t) {
        int32_t w = ((c0 + t) % M + M) % M;
        if (w == c)
            return 1;
    }
    return 0;
}

/* Pruning of the stencil (the paper's conclusions name dropping the cells
 * beyond the cutoff as future work): along an axis, cells whose indices differ
 * by a (wrapped) |t| have |t| - 1 whole cells of side L/M between them when
 * |t| >= 2, so no two of their points are closer than that gap.  A stencil cell
 * is dropped when the squared gaps, summed over the axes the stencil does not
 * cover whole, exceed rc^2 (1 + 1e-9) -- the relative margin keeps a cell whose
 * gap equals rc up to the rounding of the cell assignment.  Covered axes add
 * no gap (their offsets are not relative to the centre cell). */
static double axis_gap(int32_t at, double L, int32_t M)
{
    return at >= 2 ? (double)(at - 1) * (L / (double)M) : 0.0;
}

static int gap_beyond_cutoff(double gap2, double rc)
{
    return gap2 > rc * rc * (1.0 + 1e-9);
}

/* |t| of the offset t in [-k, k] with (c0 + t) mod M == c on an axis the
 * stencil does not cover whole, else -1. */
static int32_t axis_offset(int32_t c, int32_t c0, int32_t k, int32_t M)
{
    for (int32_t t = -k; t <= k; ++t)
        if (((c0 + t) % M + M) % M == c)
            return t < 0 ? -t : t;
    return -1;
}

/* Number of stencil cells kept for the grid of (L, rc, req_m). */
int32_t oracle_stencil_count(const double L[3], double rc, const int32_t req_m[3])
{
    int32_t M[3], k[3], span[3];
    double invS[3];
    oracle_grid(L, rc, req_m, M, invS, k, span);
    int32_t kept = 0;
    for (int32_t i = 0; i < span[0]; ++i)
        for (int32_t j = 0; j < span[1]; ++j)
            for (int32_t l = 0; l < span[2]; ++l) {
                int32_t off[3] = {i - k[0], j - k[1], l - k[2]};
                double gap2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    if (2 * k[a] + 1 >= M[a])
                        continue;
                    double g = axis_gap(off[a] < 0 ? -off[a] : off[a], L[a], M[a]);
                    gap2 += g * g;
                }
                if (!gap_beyond_cutoff(gap2, rc))
                    ++kept;
            }
    return kept;
}

/* Sorted ids j != exclude of the particles whose cell lies in the (pruned)
 * stencil of the cell of (px,py,pz).  Returns the number of ids (writes at
 * most max_out). */
int64_t oracle_neighbor_ids(int64_t n, const double* x, const double* y, const double* z,
                            double px, double py, double pz, int64_t exclude,
                            const double L[3], double rc, const int32_t req_m[3],
                            int64_t* out, int64_t max_out)
{
    int32_t M[3], k[3], span[3];
    double invS[3];
    oracle_grid(L, rc, req_m, M, invS, k, span);
    int32_t c0[3] = {axis_cell(px, invS[0], M[0]), axis_cell(py, invS[1], M[1]), axis_cell(pz, invS[2], M[2])};
    int64_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == exclude)
            continue;
        int32_t cj[3] = {axis_cell(x[j], invS[0], M[0]), axis_cell(y[j], invS[1], M[1]),
                         axis_cell(z[j], invS[2], M[2])};
        int ok = 1;
        for (int a = 0; a < 3 && ok; ++a)
            ok = in_axis_stencil(cj[a], c0[a], k[a], M[a]);
        if (ok) {
            double gap2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                if (2 * k[a] + 1 >= M[a])
                    continue;
                double g = axis_gap(axis_offset(cj[a], c0[a], k[a], M[a]), L[a], M[a]);
                gap2 += g * g;
            }
            ok = !gap_beyond_cutoff(gap2, rc);
        }
        if (ok) {
            if (cnt < max_out)
                out[cnt] = j;
            ++cnt;
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Analytic gradient of U = U_pair + U_tail (derivative of Eq. (1)).        */
/*   dU/dr_i = sum_j (24 eps / r^2) (2 s12 - s6) d_ij, d_ij = r_j - r_i     */
/*             (minimum image), s6 = (sigma^2/r^2)^3, s12 = s6^2.           */
/*   dU/deps[a][b], dU/dsig[a][b]: the derivative with respect to the       */
/*   matrix entry, each unordered pair of species types (a,b), a != b,      */
/*   contributing half to [a][b] and half to [b][a] (the derivative of U    */
/*   written with the symmetrised tables); the tail term (ordered double    */
/*   sum) contributes its (a,b) term to [a][b].  rc is held fixed.          */
/* Pairs beyond the cutoff contribute nothing (truncated potential).        */
/* ------------------------------------------------------------------------ */
static void pair_grad_terms(const oracle_params* p, int32_t a, int32_t b, double r2,
                            double* coef, double* deps, double* dsig)
{
    int ns = p->ns;
    double eps = p->eps[a * ns + b], sig = p->sigma[a * ns + b];
    *coef = 0.0; *deps = 0.0; *dsig = 0.0;
    if (!(r2 < p->rc * p->rc) || r2 == 0.0)
        return;
    double sr2 = (sig * sig) / r2;
    double s6 = sr2 * sr2 * sr2;
    double s12 = s6 * s6;
    *coef = (24.0 * eps / r2) * (2.0 * s12 - s6);
    *deps = 4.0 * (s12 - s6);
    *dsig = (4.0 * eps / sig) * (12.0 * s12 - 6.0 * s6);
}

/* Gradient of one particle's position (O(N)): gi[3]. */
void oracle_particle_gradient(int64_t n, const double* x, const double* y, const double* z, const int32_t* sp,
                              int64_t i, const oracle_params* p, double gi[3])
{
    nsum gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
    int32_t a = sp ? sp[i] : 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i)
            continue;
        double dx = oracle_min_image(x[j] - x[i], p->L[0]);
        double dy = oracle_min_image(y[j] - y[i], p->L[1]);
        double dz = oracle_min_image(z[j] - z[i], p->L[2]);
        double r2 = (dx * dx + dy * dy) + dz * dz;
        double coef, de, ds;
        pair_grad_terms(p, a, sp ? sp[j] : 0, r2, &coef, &de, &ds);
        nsum_add(&gx, coef * dx);
        nsum_add(&gy, coef * dy);
        nsum_add(&gz, coef * dz);
    }
    gi[0] = nsum_get(&gx);
    gi[1] = nsum_get(&gy);
    gi[2] = nsum_get(&gz);
}

void oracle_gradients(int64_t n, const double* x, const double* y, const double* z, const int32_t* sp,
                      const oracle_params* p, double* gx, double* gy, double* gz, double* d_eps, double* d_sig)
{
    int ns = p->ns;
    if (gx) {
        for (int64_t i = 0; i < n; ++i) {
            double g[3];
            oracle_particle_gradient(n, x, y, z, sp, i, p, g);
            gx[i] = g[0]; gy[i] = g[1]; gz[i] = g[2];
        }
    }
    nsum de[ORACLE_MAX_SPECIES * ORACLE_MAX_SPECIES], ds[ORACLE_MAX_SPECIES * ORACLE_MAX_SPECIES];
    memset(de, 0, sizeof de);
    memset(ds, 0, sizeof ds);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            int32_t a = sp ? sp[i] : 0, b = sp ? sp[j] : 0;
            double r2 = oracle_dist2(p->L, x[i], y[i], z[i], x[j], y[j], z[j]);
            double coef, e1, s1;
            pair_grad_terms(p, a, b, r2, &coef, &e1, &s1);
            if (a == b) {
                nsum_add(&de[a * ns + b], e1);
                nsum_add(&ds[a * ns + b], s1);
            } else {
                nsum_add(&de[a * ns + b], 0.5 * e1);
                nsum_add(&de[b * ns + a], 0.5 * e1);
                nsum_add(&ds[a * ns + b], 0.5 * s1);
                nsum_add(&ds[b * ns + a], 0.5 * s1);
            }
        }
    }
    int64_t counts[ORACLE_MAX_SPECIES] = {0};
    for (int64_t i = 0; i < n; ++i)
        counts[sp ? sp[i] : 0] += 1;
    double V = box_volume(p);
    for (int a = 0; a < ns; ++a) {
        for (int b = 0; b < ns; ++b) {
            double eps = p->eps[a * ns + b], sig = p->sigma[a * ns + b];
            double q = sig / p->rc;
            double q3 = q * q * q, q9 = q3 * q3 * q3;
            double pref = (8.0 * M_PI / (3.0 * V)) * (double)counts[a] * (double)counts[b];
            /* d/d eps of eps sig^3 (q^9/3 - q^3) and d/d sig of the same */
            double t_e = sig * sig * sig * (q9 / 3.0 - q3);
            double t_s = eps * (4.0 * sig * sig * q9 - 6.0 * sig * sig * q3);
            d_eps[a * ns + b] = nsum_get(&de[a * ns + b]) + pref * t_e;
            d_sig[a * ns + b] = nsum_get(&ds[a * ns + b]) + pref * t_s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pressure from the virial of the pair forces of Eq. (1).                  */
/*   w(r) = -r du/dr = 24 eps [2 (sigma/r)^12 - (sigma/r)^6]  (r < r_c)     */
/*   W    = sum over pairs i < j of w(r_ij)                                 */
/*   P    = N / (beta V) + W / (3 V) + P_tail                               */
/* P_tail is the pressure of the full potential beyond r_c, the counterpart */
/* of the energy tail correction:                                           */
/*   P_tail = -(2 pi / 3) sum_ab rho_a rho_b int_rc^inf r^3 u'_ab(r) dr     */
/*          = (16 pi / (3 V^2)) sum_ab N_a N_b eps_ab sigma_ab^3            */
/*            [(2/3) (sigma_ab/r_c)^9 - (sigma_ab/r_c)^3].                  */
/* out[0] = W, out[1] = sum |w| (tolerance scale), out[2] = P_tail,         */
/* out[3] = P.  Plain all-pairs loop, compensated sums.                     */
/* ------------------------------------------------------------------------ */
static double pair_w(const oracle_params* p, int32_t a, int32_t b, double r2)
{
    int ns = p->ns;
    double eps = p->eps[a * ns + b], sigma = p->sigma[a * ns + b];
    if (!(r2 < p->rc * p->rc) || eps == 0.0)
        return 0.0;
    if (r2 == 0.0)
        return INFINITY;
    double sr2 = (sigma * sigma) / r2;
    double sr6 = sr2 * sr2 * sr2;
    return 24.0 * eps * (2.0 * (sr6 * sr6) - sr6);
}

double oracle_tail_pressure(const int64_t* counts, const oracle_params* p)
{
    double V = box_volume(p);
    double s = 0.0;
    for (int a = 0; a < p->ns; ++a) {
        for (int b = 0; b < p->ns; ++b) {
            double eps = p->eps[a * p->ns + b], sig = p->sigma[a * p->ns + b];
            double q = sig / p->rc;
            double q3 = q * q * q;
            s += (double)counts[a] * (double)counts[b] * eps * sig * sig * sig * ((2.0 / 3.0) * q3 * q3 * q3 - q3);
        }
    }
    return (16.0 * M_PI / (3.0 * V * V)) * s;
}

void oracle_virial(int64_t n, const double* x, const double* y, const double* z, const int32_t* sp,
                   const oracle_params* p, double out[4])
{
    nsum s = {0, 0}, a = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double r2 = oracle_dist2(p->L, x[i], y[i], z[i], x[j], y[j], z[j]);
            double w = pair_w(p, sp ? sp[i] : 0, sp ? sp[j] : 0, r2);
            nsum_add(&s, w);
            nsum_add(&a, fabs(w));
        }
    }
    int64_t counts[ORACLE_MAX_SPECIES] = {0};
    for (int64_t i = 0; i < n; ++i)
        counts[sp ? sp[i] : 0] += 1;
    double V = box_volume(p);
    out[0] = nsum_get(&s);
    out[1] = nsum_get(&a);
    out[2] = oracle_tail_pressure(counts, p);
    out[3] = (double)n / (p->beta * V) + out[0] / (3.0 * V) + out[2];
}
