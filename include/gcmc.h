/*
 * gcmc.h -- C ABI of the MI355X (gfx950) grand-canonical Monte Carlo cell-list
 * library.
 *
 * The method is that of Schwiebert, Hailat, Rushaidat, Mick and Potoff, "An
 * Efficient Cell List Implementation for Monte Carlo Simulation on GPUs"
 * (arXiv 1408.3764): Lennard-Jones particles (Eq. 1) in a periodic box, trial
 * displacements, insertions and deletions accepted with the Metropolis rules of
 * Eqs. (2)-(5); each trial's energy change is the sum of the pair energies of
 * one particle with the particles in the cells around it (Sec. 3.2), split
 * across GPU threads and reduced; the cell list is updated incrementally when a
 * move is accepted (Sec. 3.2.5).
 *
 * Conventions for every entry point:
 *   - Return value: GCMC_OK (0) or a GCMC_ERR_* code; gcmc_last_error() gives a
 *     message for the calling thread.  No C++ exception crosses this boundary.
 *   - d_* arguments are DEVICE pointers owned by the caller (e.g. torch tensors),
 *     h_* arguments are HOST pointers owned by the caller.  The library owns the
 *     memory behind gcmc_box and gcmc_batch (allocated at create, freed at
 *     destroy).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     asynchronously; only gcmc_sync_status, gcmc_get_* and gcmc_export_state
 *     block.  One box may be used by one stream at a time.
 *   - Errors found on the device (a cell over capacity, N reaching max_n) are
 *     latched in the box: the offending move is NOT applied, the chain stops
 *     there, later kernels on the box do nothing, and gcmc_sync_status returns
 *     the code.  gcmc_cell_build clears it (e.g. after growing the capacity), so
 *     the chain can resume from the move counter it stopped at.
 *   - Coordinates are reduced units (sigma = epsilon = k_B = 1 for one species)
 *     and must lie in [0, L) per axis.
 */
#ifndef GCMC_H
#define GCMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GCMC_OK = 0,
    GCMC_ERR_INVALID_ARG = 1,   /* bad argument: rc > L/2, n > max_n, bad species, ... */
    GCMC_ERR_OOM = 2,           /* device allocation failed */
    GCMC_ERR_CELL_OVERFLOW = 3, /* a cell would exceed its capacity (Sec. 3.2.2: fixed-size cell arrays) */
    GCMC_ERR_CAPACITY = 4,      /* an insertion would exceed max_n */
    GCMC_ERR_HIP = 5,           /* a HIP runtime call failed */
    GCMC_ERR_POISONED = 6,      /* the box holds a latched device error */
    GCMC_ERR_UNSUPPORTED = 7,   /* valid but not implemented (e.g. a chain over a mixture) */
    GCMC_ERR_INTERNAL = 8       /* a wait inside a chain kernel (pipelined or speculative) exceeded its bound (latched; a rebuild clears it) */
};

enum { GCMC_MOVE_DISPLACE = 0, GCMC_MOVE_INSERT = 1, GCMC_MOVE_DELETE = 2 };

#define GCMC_MAX_SPECIES 4
#define GCMC_COUNTER_CONTINUE 0xFFFFFFFFFFFFFFFFull

typedef struct gcmc_box gcmc_box;
typedef struct gcmc_batch gcmc_batch;

/* Box description (host struct, copied at create).
 *   L, rc        box edges and cutoff (rc <= L_a / 2 on every axis).
 *   beta, mu     1/(k_B T) of Eq. (2) and the chemical potential of Eqs. (4)-(5).
 *   lambda3      Lambda^3 of Eqs. (4)-(5).
 *   max_disp     half-width of the uniform displacement cube.
 *   p_disp       DisplacePercent of Algorithm 1, as a fraction.
 *   n_species    1..GCMC_MAX_SPECIES; eps/sigma are HOST n_species^2 pair tables
 *                (symmetric, already mixed).
 *   max_n        particle capacity (insertions beyond it are GCMC_ERR_CAPACITY).
 *   cell_m       cells per axis, 0 = the paper's rule M = max(3, floor(L/rc))
 *                (Sec. 3.2.2); a larger M gives cells smaller than rc (the
 *                microcells of Sec. 3.3) and a wider stencil of 2k+1 cells per
 *                axis, k = ceil(rc M / L), from which the cells farther than rc
 *                from the centre cell are dropped (Sec. 5 names this pruning as
 *                future work).  At most 1024 stencil cells are kept.
 *   cell_cap     per-cell capacity, 0 = automatic.
 *   seed, box_id Philox4x32-10 key and the third counter word of the move stream. */
typedef struct {
    double L[3];
    double rc;
    double beta;
    double mu;
    double lambda3;
    double max_disp;
    double p_disp;
    int32_t n_species;
    int32_t cell_cap;
    const double* eps;
    const double* sigma;
    int64_t max_n;
    int32_t cell_m[3];
    uint32_t box_id;
    uint64_t seed;
} gcmc_box_desc;

/* One trial move for the host-driven entry points (40 bytes, device array).
 *   type     GCMC_MOVE_*.
 *   index    particle to displace or delete (0 <= index < N).
 *   x, y, z  displacement: the new position; insertion: the position; unused
 *            for deletion.  Must lie in [0, L).
 *   species  species of an inserted particle. */
typedef struct {
    int32_t type;
    int32_t index;
    double x, y, z;
    int32_t species;
    int32_t pad;
} gcmc_move;

/* Chain statistics written by gcmc_step / gcmc_batch_step (device struct),
 * one launch's worth.  The averages are the ensemble averages the paper's
 * multi-move kernel keeps on the GPU (Sec. 3.3.4: average energy and average
 * pressure), taken over the moves of the launch, each move counted with the
 * state after it; the same sums accumulated over every launch since the box
 * was created, imported or cleared are part of gcmc_checkpoint. */
typedef struct {
    int64_t attempts[3];   /* per move type */
    int64_t accepts[3];
    int64_t n;             /* N after the last move */
    int64_t moves_done;    /* moves processed (less than asked if an error stopped the chain) */
    double u_pair;         /* running pair energy after the last move */
    double u_tail;         /* tail correction at the final N */
    double sum_n;          /* sum over processed moves of N after the move */
    double sum_u;          /* sum over processed moves of u_pair + u_tail after the move */
    int32_t error;         /* GCMC_OK or the latched GCMC_ERR_* */
    int32_t pad;
    int64_t error_move;    /* move counter at which the error was raised, else -1 */
    int64_t stencils;      /* neighbour-cell stencils gathered (a same-cell displacement shares one) */
    int64_t candidates;    /* candidate particle records read from those stencils */
    int64_t pair_evals;    /* pair distances evaluated (candidates x positions evaluated against them) */
    int64_t in_cutoff;     /* of those, pairs strictly inside the cutoff */
    double w_pair;         /* running pair virial W after the last move (Sec. 3.1.2 updates the virial on
                              every acceptance; set by gcmc_virial, kept current by the chain) */
    double sum_w;          /* sum over processed moves of W after the move */
    double sum_n2;         /* sum over processed moves of N^2 after the move */
    double avg_n;          /* sum_n / moves_done (NaN if no move was processed) */
    double avg_u;          /* sum_u / moves_done */
    double avg_p;          /* average pressure N k_B T / V + W / (3V) + P_tail(N), with P_tail the
                              pressure of the potential beyond rc (as gcmc_virial), averaged over the
                              same moves: k_B T avg_n / V + (sum_w / moves) / (3V) + c (sum_n2 / moves) */
} gcmc_stats;

/* Checkpoint of a box (host struct): everything besides the particles that a
 * chain needs to continue exactly where it stopped (Algorithm 1 periodically
 * writes the system status to disk; Sec. 3.3.4 checkpoints every 10,000
 * moves).  Cumulative sums cover every move since the box was created,
 * imported or its averages cleared. */
typedef struct {
    int64_t n;             /* particles */
    double u_pair;         /* running pair energy */
    double w_pair;         /* running pair virial */
    uint64_t counter;      /* device move counter: the next move GCMC_COUNTER_CONTINUE runs */
    int64_t moves;         /* moves in the cumulative sums below */
    int64_t attempts[3];   /* per move type */
    int64_t accepts[3];
    double sum_n;          /* sums over those moves of N, N^2, u_pair + u_tail and W after each move */
    double sum_n2;
    double sum_u;
    double sum_w;
    int32_t error;         /* latched GCMC_ERR_* (export only; import needs GCMC_OK) */
    int32_t pad;
    int64_t error_move;    /* move counter of the latched error, else -1 */
} gcmc_checkpoint;

/* Optional per-move record of gcmc_step (72 bytes, device array of n_moves). */
typedef struct {
    int32_t type;      /* GCMC_MOVE_* */
    int32_t index;     /* particle index (displace/delete), new index N (insert), -1 if N == 0 */
    int32_t accepted;
    int32_t flags;     /* bit0: rejected because the box was empty */
    double dU_pair;
    double dU_tail;
    double x, y, z;    /* trial position */
    double arg;        /* log of the acceptance ratio */
    double dW_pair;    /* change of the pair virial the move would make (applied on acceptance) */
} gcmc_log;

/* Geometry chosen at create (host struct). */
typedef struct {
    int32_t cell_m[3];   /* cells per axis */
    int32_t span[3];     /* stencil cells per axis */
    int32_t cell_cap;    /* per-cell capacity */
    int32_t n_species;
    int64_t n_cells;
    int64_t max_n;
    double inv_s[3];     /* M_a / L_a */
    int32_t n_stencil;   /* stencil cells kept: the span_x x span_y x span_z block less
                            the cells whose closest point to the centre cell lies
                            beyond rc (dropped only on axes not covered whole) */
    int32_t pad;
} gcmc_box_info;

/* ---------------------------------------------------------------- boxes */

/* Create a box from n particles given as device SoA arrays (d_species may be
 * NULL for one species) and bin them into the cell list (the initial binning of
 * Sec. 3.2.1, atomic slot claims, then a per-cell ordering by particle index so
 * the layout is deterministic).  Blocks until the binning is done so that an
 * overflow is reported here.  *out receives the box. */
int gcmc_box_create(const gcmc_box_desc* desc, const double* d_x, const double* d_y, const double* d_z,
                    const int32_t* d_species, int64_t n, void* stream, gcmc_box** out);
/* Release a box (the device arrays of Sec. 3.2.1's cell list and the particle
 * records).  Waits for the device first; the handle is invalid afterwards. */
int gcmc_box_destroy(gcmc_box* box);
/* The cell grid chosen at create (Sec. 3.2.2: cells per axis, stencil). */
int gcmc_box_get_info(const gcmc_box* box, gcmc_box_info* h_info);

/* Re-bin the current particles (Sec. 3.2.1), optionally with a new per-cell
 * capacity (new_cap > 0 reallocates).  Clears a latched cell-overflow or
 * wait-bound (GCMC_ERR_INTERNAL) error: both stop the chain before a move with
 * every earlier move committed, so it can resume at its error_move counter. */
int gcmc_cell_build(gcmc_box* box, int32_t new_cap, void* stream);

/* Replace the positions of the current particles and re-bin (Sec. 3.2.1);
 * used by the autograd wrapper between forward passes (Eq. 1 evaluated at new
 * coordinates).  n must equal the box's N (else GCMC_ERR_INVALID_ARG and
 * nothing changes): d_x, d_y, d_z hold n coordinates each, in [0, L).
 * Species, the move counter and the cumulative sums are kept.  The running
 * pair energy and virial no longer describe the configuration: both become
 * NaN until gcmc_total_energy and gcmc_virial set them again. */
int gcmc_set_positions(gcmc_box* box, const double* d_x, const double* d_y, const double* d_z, int64_t n,
                       void* stream);

/* Volume change (the cell-list rebuild and total energy that volume moves of
 * the Gibbs ensemble need, proposed in the conclusions, Sec. 5): every
 * coordinate is scaled by L'_a / L_a (x -> x * (L'_a / L_a), the ratio rounded
 * once, kept in [0, L'_a)), the cell grid is rebuilt for the new edges by the
 * box's rule (the cell_m given at create, else max(3, floor(L'/rc))), the
 * tail-correction constants follow the new volume, the cell capacity grows by
 * the creation rule if the densest new cell needs it, and particles are
 * re-binned (same indices, species and move counter).  h_L: HOST array of the
 * three new edges (> 0, rc <= L'_a / 2; else GCMC_ERR_INVALID_ARG and nothing
 * changes).  d_U: DEVICE array of 4 doubles written with the cell-list
 * U_pair and U_tail at the new volume, then at the old one; the box's running
 * pair energy is reset to the new U_pair (as gcmc_total_energy does).  A box
 * holding a latched error
 * is refused (GCMC_ERR_POISONED).  Blocks the host until done; an allocation
 * failure after the coordinates were scaled leaves the box unusable. */
int gcmc_box_rescale(gcmc_box* box, const double* h_L, double* d_U, void* stream);

/* Replace the force field (the eps_ab, sigma_ab of Eq. 1): h_eps, h_sigma are
 * HOST n_species^2 pair tables (symmetric, eps >= 0, sigma > 0), as in
 * gcmc_box_desc.  Blocks until work already queued on the box is done.  The
 * running pair energy and virial become NaN until gcmc_total_energy and
 * gcmc_virial set them for the new force field. */
int gcmc_set_params(gcmc_box* box, const double* h_eps, const double* h_sigma);

/* ------------------------------------------------------------ the moves */

/* Energy change of n_moves independent trial moves against the current
 * configuration, no commit (the per-move energy of Algorithms 6 and 7: the
 * stencil cells around the old and/or new position, one candidate per lane,
 * wavefront then workgroup reduction).  d_moves[n_moves] as gcmc_move;
 * d_dU_pair[n_moves] receives the pair part (displacement: new - old;
 * insertion: + energy at the point; deletion: - energy of the particle);
 * d_dU_tail[n_moves] (may be NULL) the tail-correction change; d_dW_pair
 * [n_moves] (may be NULL) the change of the pair virial W (the sum of
 * 24 eps [2 (sigma/r)^12 - (sigma/r)^6] over pairs inside the cutoff), which
 * Sec. 3.1.2 updates with the energy on acceptance.  A move with a bad index
 * or species gives NaN. */
int gcmc_delta_energy(gcmc_box* box, const gcmc_move* d_moves, int64_t n_moves, double* d_dU_pair,
                      double* d_dU_tail, double* d_dW_pair, void* stream);

/* The same quantities over all N particles, without the cell list (the
 * no-cell-list path of Algorithms 3 and 4): many workgroups per move, partial
 * sums reduced by a second kernel in a fixed order. */
int gcmc_delta_energy_allpairs(gcmc_box* box, const gcmc_move* d_moves, int64_t n_moves, double* d_dU_pair,
                               double* d_dU_tail, double* d_dW_pair, void* stream);

/* Apply one accepted move (device gcmc_move) whose pair-energy change is
 * *d_dU_pair and pair-virial change *d_dW_pair (as returned by
 * gcmc_delta_energy): position write, N +- 1, the running pair energy and
 * virial (an accepted move updates both, Sec. 3.1.2), and the incremental
 * cell update of Sec. 3.2.5
 * (remove from the old cell by swapping in the cell's last entry, append to
 * the new cell; nothing when the cell is unchanged); a deletion moves particle
 * N-1 to the freed index.  d_dW_pair may be NULL: the running virial then
 * becomes NaN until gcmc_virial sets it. */
int gcmc_commit(gcmc_box* box, const gcmc_move* d_move, const double* d_dU_pair, const double* d_dW_pair,
                void* stream);

/* Launch shape of the chain kernels (the autotuner's choice).  rows > 0: one
 * move at a time, `waves` wavefronts per workgroup and `rows` candidate slots
 * per lane per pass (1x8, 2x8, 4x2, 4x4, 4x8, 8x2, 8x4).  rows = 0:
 * speculative rounds, `waves` (2, 4, 8 or 16) consecutive moves evaluated at once,
 * one per wavefront, against the round's starting state and committed in
 * order, each only if nothing it read has changed since (the same chain, move
 * for move); needs one species and at most 512 stencil cells (stencils of
 * more than 32 cells, or whose candidates exceed 8192 slots, go through a
 * path that loads the stencil counters in groups of 64 cells and stages the
 * candidates' record indices in LDS windows), else GCMC_ERR_UNSUPPORTED.
 * rows = -1: pipelined, one wavefront decides the moves in order while
 * waves - 1 (3 or 7) wavefronts evaluate the moves ahead of it; an evaluation
 * is used only if no decision since it read memory changed what it read (the
 * same chain, move for move); needs one species, at most 32 stencil cells,
 * 2 x stencil cells x cell_cap <= 8192 and at most 1024 cells per axis.
 * rows = -2:
 * the paper's microcell thread mapping (Sec. 3.3.2), one move at a time, each
 * thread of `waves` (4 or 8) wavefronts taking one stencil cell (several when
 * the stencil is larger) and looping over the particles in it; any grid.
 * rows = -3: the box held in LDS (for small boxes, Sec. 5's many simulations
 * on one GPU): the coordinates of particles 0 .. 2047 are copied into the
 * workgroup's local memory once per launch; rounds of `waves` (4 or 8) moves
 * are evaluated against every other particle (the pairs inside the cutoff are
 * the ones the cell list finds) and decided in order, each corrected for the
 * earlier accepted moves of its round (the same chain, move for move);
 * particles past 2047 stay in global memory (correct, slower).  The cell list is not updated during the launch; at its end it is
 * rebuilt in gcmc_cell_build's layout (a cell that overflows latches
 * GCMC_ERR_CELL_OVERFLOW after the launch's last move, and a rebuild with a
 * larger capacity clears it).  One species. */
int gcmc_box_set_launch(gcmc_box* box, int32_t waves, int32_t rows);

/* Bound on the in-kernel waits of the speculative and pipelined chains (a
 * wavefront polling an LDS flag that another wavefront of its workgroup sets;
 * no such wait depends on another workgroup or on the host).  polls > 0: a
 * wait gives up after that many polls; 0: the default, 2^26 polls (seconds);
 * < 0: every wait gives up at once, so a launch that reaches one stops there
 * with GCMC_ERR_INTERNAL latched (the chain stops before the waiting move, as
 * on a cell overflow, and gcmc_cell_build clears it).  For tests of that error path; the per-move chain has
 * no such waits.  Blocks until work already queued on the box is done; batches
 * take the value of each box. */
int gcmc_box_set_wait_limit(gcmc_box* box, int32_t polls);

/* Run n_moves moves of the Markov chain of Algorithm 1 on the device in one
 * persistent launch (Sec. 3.3.4: one kernel call for many moves): move m uses
 * the Philox4x32-10 stream with key = seed and counter
 * (counter0 + m low, high, box_id, j), j = 0..3, giving eight uniforms
 * (R, Source, particle pick u2, A, three position draws, pick fields u7);
 * R < p_disp is a displacement, else Source < 0.5 a deletion, else an
 * insertion.  A displacement or deletion among N particles takes the first
 * b-bit field of u7's 53 bits (u7 = k 2^-53, high field first, 2^b the
 * smallest power of two >= N) whose value is below N, else min(floor(u2 N),
 * N - 1): Algorithm 2's random particle, uniform over 0 .. N-1.  Single
 * species only.  counter0 = GCMC_COUNTER_CONTINUE starts at the box's device
 * counter (the move after the last one run), so a captured HIP graph of
 * gcmc_step calls continues the chain each time it is replayed.  d_stats (may
 * be NULL) receives the chain statistics and d_log (may be NULL) one record per
 * move. */
int gcmc_step(gcmc_box* box, int64_t n_moves, uint64_t counter0, gcmc_stats* d_stats, gcmc_log* d_log,
              void* stream);

/* The same chain with every energy computed over all particles (no cell
 * list), two launches per move (evaluate over many workgroups; reduce, decide
 * and commit in one), for comparison with gcmc_step. */
int gcmc_step_allpairs(gcmc_box* box, int64_t n_moves, uint64_t counter0, gcmc_stats* d_stats,
                       gcmc_log* d_log, void* stream);

/* --------------------------------------------------------- total energy */

/* Total energy (Sec. 3.1.1): d_U[0] = U_pair = (1/2) sum_i e_i over the cell
 * stencils (all_pairs = 0) or over all pairs (all_pairs = 1), d_U[1] = U_tail.
 * d_e[N] (may be NULL) receives e_i = sum_{j != i} u(r_ij) in particle order.
 * Also resets the running energy of the chain to d_U[0]. */
int gcmc_total_energy(gcmc_box* box, int32_t all_pairs, double* d_U, double* d_e, void* stream);

/* gcmc_total_energy for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same kernels,
 * the same results bit for bit, with the pass's scratch in a 16 MiB array
 * (2^21 doubles) that the library holds per GPU until the process ends
 * instead of the box's scratch.  A pass over the cell list needs about
 * N / 256 + (N + cells) / 2 doubles, so N + cells up to about 4.1 million
 * fit; a larger box is refused with GCMC_ERR_INVALID_ARG (nothing launched).
 * Calls no allocating routine.  It still reads the box state back to the host
 * (as gcmc_total_energy does), so it blocks on `stream`.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  The current
 * device must be the box's. */
int gcmc_total_energy_noalloc(gcmc_box* box, int32_t all_pairs, double* d_U, double* d_e, void* stream);

/* Gradient of U = U_pair + U_tail (Eq. 1 differentiated; rc held fixed):
 * d_grad[3*N] (SoA: x block, y block, z block) = dU/dr_i; d_deps and d_dsig
 * [n_species^2] = dU/d eps_ab and dU/d sigma_ab, where an unordered species
 * pair a != b contributes half to [a][b] and half to [b][a].  Any of the three
 * outputs may be NULL. */
int gcmc_backward(gcmc_box* box, double* d_grad, double* d_deps, double* d_dsig, void* stream);

/* Pressure from the virial of the pair forces (Eq. 1 differentiated, as in
 * gcmc_backward; the running averages of the chain are in gcmc_stats).
 * d_out[0] = W = sum over pairs inside the cutoff of -r du/dr
 *              = sum 24 eps_ab [2 (sigma_ab/r)^12 - (sigma_ab/r)^6],
 * d_out[1] = P = N k_B T / V + W / (3 V) + P_tail, where P_tail is the
 * pressure of the full potential beyond r_c (the counterpart of U_tail):
 * (16 pi / (3 V^2)) sum_ab N_a N_b eps_ab sigma_ab^3 [(2/3)(sigma_ab/r_c)^9
 * - (sigma_ab/r_c)^3].  Cell-list sums in a fixed order; d_out is device
 * memory, written on `stream`.  Also sets the running pair virial that the
 * chain keeps current on every acceptance (Sec. 3.1.2) to W. */
int gcmc_virial(gcmc_box* box, double* d_out, void* stream);

/* ------------------------------------------------------------- batches */

/* Group existing single-species boxes (all must stay alive) so that
 * gcmc_batch_step advances all of them in one persistent launch: the paper's
 * conclusions (Sec. 5) note that one microcell chain uses a single
 * multiprocessor, leaving room to run many simulations on one GPU at once.
 * One workgroup per box, boxes ordered by decreasing N; each box keeps its own
 * launch shape (gcmc_box_set_launch), and boxes of different shapes go to
 * separate launches on the same stream.  boxes[n_boxes] is a HOST array of
 * handles, copied. */
int gcmc_batch_create(gcmc_box* const* boxes, int32_t n_boxes, gcmc_batch** out);
/* Release a batch (not its boxes). */
int gcmc_batch_destroy(gcmc_batch* batch);
/* Advance every box of the batch by moves_per_box moves (counter0 + m, the
 * box's own box_id and seed; GCMC_COUNTER_CONTINUE: each box's device
 * counter).  d_stats[n_boxes] (may be NULL), in the order the boxes were
 * given.  Boxes are grouped by their launch path and shape (at most 8
 * groups): one kernel per group, the first on `stream`, the others on side
 * streams of the batch forked from `stream` and joined back to it with
 * events, so the groups run at the same time and everything is ordered on
 * `stream`.  No host synchronisation, so it can be captured in a HIP graph,
 * except on the first call and after a box was rebuilt or its launch shape
 * changed: that call re-uploads the descriptors and, for several groups,
 * creates the side streams and events. */
int gcmc_batch_step(gcmc_batch* batch, int64_t moves_per_box, uint64_t counter0, gcmc_stats* d_stats,
                    void* stream);

/* ---------------------------------------------------- inspection / state */

/* Copy the current particles out (blocks): d_x, d_y, d_z [>= N] (may be NULL),
 * d_species [>= N] (may be NULL); *h_n receives N. */
int gcmc_get_particles(gcmc_box* box, double* d_x, double* d_y, double* d_z, int32_t* d_species, int64_t* h_n,
                       void* stream);

/* Copy the cell list out (blocks), the ParticlesInCells arrays of Sec. 3.2.1:
 * d_cell_of[N] the cell of each particle, d_count[n_cells] the per-cell
 * counters, d_ids[n_cells * cell_cap] cell-major particle ids (entries past a
 * cell's count are unspecified).  Any pointer may be NULL. */
int gcmc_get_cells(gcmc_box* box, int32_t* d_cell_of, int32_t* d_count, int32_t* d_ids, void* stream);

/* Neighbour candidates (the particles in the stencil cells of a point, the
 * moving particle excluded) of n points, gathered by the same device code as
 * the energy kernels.  d_points[3*n] SoA (x block, y, z), d_exclude[n] (id or
 * -1), d_ids[n * max_ids] receives the ids in unspecified order, d_counts[n]
 * the full count (ids beyond max_ids are dropped). */
int gcmc_neighbor_ids(gcmc_box* box, const double* d_points, const int32_t* d_exclude, int64_t n,
                      int32_t max_ids, int32_t* d_ids, int32_t* d_counts, void* stream);

/* Checkpoint (blocks after the work queued on `stream`): the periodic
 * system-status dump of Algorithm 1, taken every so many moves (Sec. 3.3.4).
 * h_ck receives N, the running energy and virial, the device move counter,
 * the cumulative statistics and the latched error.  d_x, d_y, d_z, d_species
 * (device, each may be NULL) receive the N particles; `capacity` is their
 * length (GCMC_ERR_INVALID_ARG if a pointer is given and capacity < N). */
int gcmc_export_state(gcmc_box* box, double* d_x, double* d_y, double* d_z, int32_t* d_species, int64_t capacity,
                      gcmc_checkpoint* h_ck, void* stream);
/* Restore a checkpoint into a box with the same geometry and force field:
 * h_ck->n particles from device SoA arrays (d_species may be NULL for one
 * species; n <= max_n), the running energy and virial, the move counter and
 * the cumulative statistics, then re-bin (Sec. 3.2.1).  A chain continued
 * with GCMC_COUNTER_CONTINUE is then the uninterrupted chain.  h_ck->error must
 * be GCMC_OK (GCMC_ERR_INVALID_ARG otherwise). */
int gcmc_import_state(gcmc_box* box, const double* d_x, const double* d_y, const double* d_z,
                      const int32_t* d_species, const gcmc_checkpoint* h_ck, void* stream);
/* Zero the cumulative statistics of the checkpoint (e.g. after equilibration);
 * the running energy, virial and move counter are kept.  Enqueued on
 * `stream`. */
int gcmc_clear_averages(gcmc_box* box, void* stream);

/* Block until the box's queued work is done; returns its latched error (a
 * device error of the kind the paper's kernels would report to the host after
 * a move: cell over capacity, N at max_n). */
int gcmc_sync_status(gcmc_box* box);

/* Message for the last error on the calling thread ("" if none): the text
 * behind the GCMC_ERR_* code of the call that failed last. */
const char* gcmc_last_error(void);

/* Library version string. */
const char* gcmc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GCMC_H */
