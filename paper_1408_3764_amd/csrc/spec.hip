// Speculative evaluation of consecutive moves of one chain, committed in order
// (the exact chain of Algorithm 1; not the "keep the first accepted" scheme the
// paper lists as future work, which would change the sampled distribution).
//
// A round takes the next W moves.  Wavefront w evaluates move m + w against
// the state at the start of the round:
//   * its Philox draws, type and trial positions.  A displacement or deletion
//     picks floor(u N), which moves with N: the wavefront also computes the
//     draws of the earlier moves of the round, so it knows how many insertions
//     and deletions precede its move, and evaluates the pick at the N expected
//     at its commit from the chain's running acceptance rates;
//   * the counters of its stencil cells (one lane per cell, both stencils of a
//     displacement that leaves its cell: at most 64 cells), an in-wave prefix
//     sum of the counters, an owner table in LDS mapping each flattened
//     candidate to its cell, and then exactly the candidates' 32-byte records
//     (one memory round trip for the counters, one for the records);
//   * the pair sums, reduced across the wavefront, and ln A.
// Wavefront 0 then walks the round's moves in order, taking each as soon as
// its wavefront has published it (a flag in LDS), while slower wavefronts may
// still be evaluating.  A move's evaluation is
// used only if nothing it read has changed since the round started: its pick
// at the current N is the one it evaluated, the particle record
// it read was not touched by an earlier commit of the round, and no cell
// modified by an earlier commit lies in one of its stencils.  Then the tail
// correction and the acceptance prefactor are taken at the current N, the
// Metropolis test is applied and an accepted move is committed (stores only;
// the records it needs came back with its evaluation).  N moves by at most one
// per move, so the records of particles N_round - W .. N_round + W - 1 (what a
// deletion moves into the freed index) and the prefactors for those N are
// prepared in LDS by wavefront 0 at the start of the round, and kept current by
// the commits.  The check also covers commits whose stores land while a later
// move is still reading: whatever a commit writes lies in a modified cell or a
// touched particle record.  The first move that
// fails the check ends the round and is evaluated again in the next one, so
// every move is decided on exactly the state the sequential chain would have.
//
// NG > 0: stencils of more than 32 cells (microcells, Sec. 3.3) go through
// the evaluation's path with NG groups of 64 cells; the round and the commit
// are the same.
#include "spec_eval.h"

namespace gcmc {

// Tail change and log acceptance ratio of a move decided at N particles
// (Eqs. 3-5; the log prefactors for N come from the round's tables): one
// routine for the decision and for the per-move log written after the round,
// so both hold the same bits.
// The parts of it that do not depend on the evaluation (the tail change and the log
// prefactor at N), and the rest; the decision and the per-move log both go through them.
__device__ __forceinline__ void spec_arg_pre(int type, int64_t N, int64_t base, const double* lp_ins,
                                             const double* lp_del, double tk, double& dUt, double& lpref) {
    const bool is_disp = type == GCMC_MOVE_DISPLACE, is_ins = type == GCMC_MOVE_INSERT;
    dUt = is_disp ? 0.0 : tk * (is_ins ? (2.0 * (double)N + 1.0) : (1.0 - 2.0 * (double)N));
    lpref = is_disp ? 0.0 : (is_ins ? lp_ins[N - base] : lp_del[N - base]);
}

__device__ __forceinline__ double spec_arg_fin(const DevBox& B, int type, double dUp, double dUt, double lpref) {
    const bool is_disp = type == GCMC_MOVE_DISPLACE, is_ins = type == GCMC_MOVE_INSERT;
    const double dU = dUp + dUt;
    return is_disp ? -(B.beta * dU) : (is_ins ? lpref + B.beta * (B.mu - dU) : lpref - B.beta * (B.mu + dU));
}

__device__ __forceinline__ double spec_arg(const DevBox& B, int type, double dUp, int64_t N, int64_t base,
                                           const double* lp_ins, const double* lp_del, double tk, double& dUt) {
    double lpref;
    spec_arg_pre(type, N, base, lp_ins, lp_del, tk, dUt, lpref);
    return spec_arg_fin(B, type, dUp, dUt, lpref);
}

// Entry t of a prefactor table starting at N = nb: t < 4W, the log insertion
// prefactor V / (Lambda^3 (N + 1)) at N = nb + t; t >= 4W, the log deletion
// prefactor Lambda^3 N / V at N = nb + t - 4W (entries at N < 0 are never read).
template <int W>
__device__ __forceinline__ void spec_prefactor(const DevBox& B, double* lpi, double* lpd, int64_t nb, int t) {
    const bool del = t >= 4 * W;
    const int64_t n = nb + (del ? t - 4 * W : t);
    const double x = del ? (B.lambda3 * (double)n) / B.V : B.V / (B.lambda3 * (double)(n + 1));
    const double lx = log(x);
    if (del) lpd[t - 4 * W] = lx;
    else lpi[t] = lx;
}

template <int W, int CR, int NG>
__global__ __launch_bounds__(kWave* W) void k_chain_spec(const DevBox* __restrict__ boxes,
                                                          const int32_t* __restrict__ order, int64_t n_moves,
                                                          uint64_t ctr0, gcmc_stats* stats, gcmc_log* trace) {
    constexpr int kOffs = NG ? NG * kWave / 2 : 64;    // stencil slots with a precomputed linear offset
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ int32_t offs[kOffs];
    __shared__ SpecRec recs[W];
    __shared__ __align__(8) uint32_t own[W][spec_own_words(NG)];   // cell bases and start masks, or record indices
    __shared__ double4 top[2 * W];              // records of particles base .. base + 2W - 1
    // log acceptance prefactors at N = lp_base[b] + t, t < 4W, two buffers: the round's and the next round's
    __shared__ double lp_ins[2][4 * W], lp_del[2][4 * W];
    __shared__ int64_t lp_base[2];
    __shared__ DrawRing<2 * W> dring;           // draws of moves m .. m + 2W - 1
    __shared__ double pq[W][kPairRing];         // each wavefront's queue of in-cutoff pairs
    __shared__ int32_t ticket;                  // round whose next-round tables a wavefront has taken on
    __shared__ int64_t sh_state[4];       // N, moves done, error, error move
    __shared__ double sh_u, sh_w;
    __shared__ double sh_acc[2];
    __shared__ int32_t sh_maxc;
    __shared__ int32_t ready[W];                // round whose evaluation wavefront w has published
    __shared__ int64_t after_n[W];              // N, U and W after each move decided this round
    __shared__ double after_u[W], after_w[W];
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;
    const DevBox B = hot_copy(boxes[blockIdx.x]);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    BoxState* st = B.st;

    if (ctr0 == GCMC_COUNTER_CONTINUE) ctr0 = (uint64_t)st->counter;
    int64_t N = st->n;
    double U = st->u_pair;
    double Wvir = st->w_pair;
    int32_t maxc = st->maxcount;
    int32_t err = st->error;
    int64_t err_move = st->error_move;
    const double tk = B.tailK[0];
    const int cap = B.cap;
    const bool no_full = !(B.full[0] | B.full[1] | B.full[2]);
    const int32_t spin_cap = wait_bound(B.wait_limit);
    // statistics (wavefront 0 keeps them): attempts and acceptances per move type as separate
    // doubles (a dynamically indexed array would live in scratch; exact below 2^53), folded in
    // once per round
    double att0 = 0.0, att1 = 0.0, att2 = 0.0, acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    // per-lane sums over the moves lane j decided (N, N^2, U + U_tail, W after move j of a round)
    double sum_n = 0.0, sum_u = 0.0, sum_n2 = 0.0, sum_w = 0.0;
    // per-lane sums over the moves lane j decided as move j of a round, added up at the end
    int64_t stencils = 0, cand = 0, evals = 0, incut = 0;
    for (int t = tid; t < B.nstencil; t += blockDim.x) {
        const uint32_t pk = gload(B.stab + t);
        const int tx = pk & 0x3FF, ty = (pk >> 10) & 0x3FF, tz = pk >> 20;
        tab[t] = pk;
        if (t < kOffs) offs[t] = ((tz - B.k[2]) * B.M[1] + (ty - B.k[1])) * B.M[0] + (tx - B.k[0]);
    }
    if (tid < W) ready[tid] = -1;
    if (tid == 0) ticket = 0;
    // draws of the first 2W moves and the prefactors of the first round (its buffer: 1)
    for (int t = tid; t < 8 * W; t += blockDim.x) draw_block(B, &dring, ctr0 + (uint64_t)(t >> 2), t & 3);
    for (int t = tid; t < 8 * W; t += blockDim.x) spec_prefactor<W>(B, lp_ins[1], lp_del[1], N - 2 * W, t);
    if (tid == 0) lp_base[1] = N - 2 * W;
    __syncthreads();
    if (err == GCMC_OK && B.ns != 1) {
        err = GCMC_ERR_UNSUPPORTED;
        err_move = (int64_t)ctr0;
    }
    int64_t m = 0;
    int32_t rnd = 0;                   // rounds begun
    double a_ins = 0.5, a_del = 0.5;   // running acceptance of insertions and deletions
    while (err == GCMC_OK && m < n_moves) {
        const int64_t base = N - W;
        rnd = rnd == INT32_MAX ? 1 : rnd + 1;   // round numbers stay positive (a flag starts at -1)
        // issue priority on each SIMD: the moves decided first evaluate first (the two
        // wavefronts sharing a SIMD are w and w + 4 when W = 8); wavefront 0 raises its own
        // for the commit
        if (wv < (W + 1) / 2) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(1);
        // the round's prefactor table (filled before the round began)
        const int tb = rnd & 1;
        const int64_t lbase = lp_base[tb];
        const double* lpi = lp_ins[tb];
        const double* lpd = lp_del[tb];
        // ------------------------------------------------ the round's particle records (wavefront 0 commits with them)
        double4 tv = make_double4(0, 0, 0, 0);
        if (wv == 0 && lane < W && base + lane >= 0) tv = gload(B.pos + base + lane);
        // ------------------------------------------------ evaluate W moves
        if (m + wv < n_moves) {
            SpecKey key;
            // what the decision at every N the move can meet (within W - 1 of the round's N; lane o
            // takes N - (W - 1) + o) needs before the evaluation ends: the pick still the evaluated
            // one, the tail change and the prefactor -- computed while the picked record is loaded
            const int64_t np = N - (W - 1) + lane;
            const bool lane_n = lane < 2 * W - 1 && np >= 0;
            bool pick_ok = false;
            double dUt = 0.0, lpref = 0.0;
            auto early = [&](int type, double u2, double u7, int64_t idx) {
                if (lane_n) {
                    pick_ok = type == GCMC_MOVE_INSERT || spec_pick(u2, u7, np) == idx;
                    spec_arg_pre(type, np, lbase, lpi, lpd, tk, dUt, lpref);
                }
            };
            spec_eval<CR, NG, 2 * W>(B, tab, offs, own[wv], pq[wv], &dring, ctr0 + (uint64_t)m, wv, N, no_full, a_ins,
                                     a_del, &recs[wv], key, early);
            // the Metropolis test (Eqs. 3-5) at each of those N -- the operations the commit would
            // do, so the commit only reads the bit of its N
            if (!(key.flags & 1)) {
                bool acc = false;
                if (lane_n) {
                    const double arg = spec_arg_fin(B, key.type, key.dUp, dUt, lpref);
                    const double dU = key.dUp + dUt;
                    acc = dU == dU && key.lnA < arg;
                }
                const uint64_t pm = __ballot(pick_ok), am = __ballot(acc);
                if (lane == 0) {
                    recs[wv].pickmask = (uint32_t)pm;
                    recs[wv].okmask = (uint32_t)am;
                }
            }
        }
        if (wv != 0) {
            // publish this move's record: wavefront 0 decides it as soon as its turn comes, while
            // slower wavefronts still evaluate.  A commit may then store to memory that a later
            // move of the round is still reading; such a move fails the in-order check (its
            // stencil holds a modified cell, or its particle was touched) and is discarded.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            if (lane == 0) __hip_atomic_store(&ready[wv], rnd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_s_setprio(0);
            // the first wavefront to publish prepares the next round's tables while the others
            // still evaluate: the draws of moves m + W .. m + 2W - 1 (the next round takes moves
            // m + k .. m + k + W - 1 with 1 <= k <= W; the others are in the ring already) and
            // the prefactors for every N the next round can reach (within 2W - 1 of this
            // round's N).  The barrier at the end of the round makes them visible.
            int32_t prev = 0;
            if (lane == 0) prev = __hip_atomic_exchange(&ticket, rnd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (__builtin_amdgcn_readfirstlane(prev) != rnd) {
                if (lane < 4 * W)
                    draw_block(B, &dring, ctr0 + (uint64_t)(m + W) + (uint64_t)(lane >> 2), lane & 3);
                for (int t = lane; t < 8 * W; t += kWave) spec_prefactor<W>(B, lp_ins[tb ^ 1], lp_del[tb ^ 1], N - 2 * W, t);
                if (lane == 0) lp_base[tb ^ 1] = N - 2 * W;
            }
        }
        // ------------------------------------------------ in-order commit
        if (wv == 0) {
            __builtin_amdgcn_s_setprio(3);
            if (lane < W && base + lane >= 0) top[lane] = tv;
            // this wavefront's own table and record writes, seen by all of its lanes
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup", "local");
            const int64_t n_round = N;   // N at the round's start: the masks' reference
            int32_t modx = 0, mody = 0, modz = 0, touched = -1;   // lane-held lists of this round
            int nmod = 0, ntouch = 0;
            uint64_t okbits = 0;   // bit k: move k of the round accepted
            int k = 0;
            const int kend = (n_moves - m) < W ? (int)(n_moves - m) : W;
            for (; k < kend; ++k) {
                const uint64_t ctr = ctr0 + (uint64_t)(m + k);
                if (k > 0) {
                    // wait for wavefront k's evaluation (bounded: it publishes without waiting on anything)
                    int32_t spins = 0;
                    while (uni(__hip_atomic_load(&ready[k], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) != rnd) {
                        __builtin_amdgcn_s_sleep(1);
                        if (++spins > spin_cap) break;
                    }
                    if (spins > spin_cap) {
                        err = GCMC_ERR_INTERNAL;
                        err_move = (int64_t)ctr;
                        break;
                    }
                }
                const SpecRec& R = recs[k];
                // what every decision reads, loaded together (one LDS round trip, not one per test)
                const int32_t r_type = R.type, r_flags = R.flags;
                const uint32_t r_pm = R.pickmask, r_om = R.okmask;
                const int64_t r_idx = R.idx;
                int32_t cc[3] = {R.c0[0], R.c0[1], R.c0[2]};
                int32_t cn[3] = {R.c1[0], R.c1[1], R.c1[2]};
                asm volatile("" ::"v"(r_type), "v"(r_flags), "v"(r_pm), "v"(r_om), "v"(r_idx), "v"(cc[0]), "v"(cc[1]),
                             "v"(cc[2]), "v"(cn[0]), "v"(cn[1]), "v"(cn[2]));
                const int type = __builtin_amdgcn_readfirstlane(r_type);
                // the empty-box rejection holds only while the box is still empty
                if (r_flags & 1) {
                    if (N != 0) break;
                    if (lane == 0) {
                        after_n[k] = N;
                        after_u[k] = U;
                        after_w[k] = Wvir;
                    }
                    continue;
                }
                const int64_t idx = r_idx;
                const int o = (int)(N - n_round) + (W - 1);   // 0 .. 2W - 2 (N moved by at most k < W)
                if (type != GCMC_MOVE_INSERT) {
                    if (((r_pm >> o) & 1u) == 0) break;
                    if (__ballot(lane < ntouch && touched == (int32_t)idx) != 0) break;
                }
                // a cell changed by an earlier commit of this round inside one of its stencils
                bool hit = false;
                if (lane < nmod)
                    hit = in_stencil(B, modx, mody, modz, cc) ||
                          (type == GCMC_MOVE_DISPLACE && in_stencil(B, modx, mody, modz, cn));
                if (__ballot(hit) != 0) break;
                // ---- decide at the current N
                const bool is_disp = type == GCMC_MOVE_DISPLACE, is_ins = type == GCMC_MOVE_INSERT;
                const bool ok = ((r_om >> o) & 1u) != 0;
                const int two = R.two;
                const int32_t cnt0 = R.cnt0, cnt1 = R.cnt1;
                if (ok) {
                    int e = GCMC_OK;
                    if (is_ins) {
                        if (N >= B.max_n) e = GCMC_ERR_CAPACITY;
                        else if (cnt0 >= cap) e = GCMC_ERR_CELL_OVERFLOW;
                    } else if (is_disp && two) {
                        if (cnt1 >= cap) e = GCMC_ERR_CELL_OVERFLOW;
                    }
                    if (e != GCMC_OK) {
                        err = e;
                        err_move = (int64_t)ctr;
                        break;
                    }
                    // slot and cell indices fit 32 bits (cells x capacity < 2^31 for this kernel)
                    const int32_t loc = meta_low(R.rec.w);
                    const int32_t c0 = R.cl0, c1 = R.cl1;
                    const bool removes = (type == GCMC_MOVE_DELETE) || (is_disp && two);
                    const int32_t last = c0 * cap + cnt0 - 1;
                    const bool swap = removes && loc != last;
                    const int32_t id_last = swap ? meta_low(R.elast.w) : -1;
                    // the record of particle N-1 as of now (kept as scalars so that it stays in registers)
                    double rlx = 0.0, rly = 0.0, rlz = 0.0, rlw = 0.0;
                    if (type == GCMC_MOVE_DELETE) {
                        const double4 v = top[N - 1 - base];
                        rlx = v.x; rly = v.y; rlz = v.z; rlw = v.w;
                    }
                    if (lane == 0) {
                        // every store to pos[j] for j in the round's window is mirrored in top[]
                        if (swap) {
                            gstore(B.ent + loc, R.elast);
                            const double w = pack_meta(meta_species(R.elast.w), (int32_t)loc);
                            gstore_w(B.pos + id_last, w);
                            const int64_t t = (int64_t)id_last - base;
                            if (t >= 0 && t < 2 * W) top[t].w = w;
                        }
                        if (removes) gstore(B.count + c0, cnt0 - 1);
                        double4 nr;
                        int64_t j = -1;
                        if (is_disp) {
                            if (!two) {
                                gstore(B.ent + loc, make_double4(R.p1[0], R.p1[1], R.p1[2], pack_meta(0, (int32_t)idx)));
                                nr = make_double4(R.p1[0], R.p1[1], R.p1[2], R.rec.w);
                            } else {
                                const int32_t nl = c1 * cap + cnt1;
                                gstore(B.ent + nl, make_double4(R.p1[0], R.p1[1], R.p1[2], pack_meta(0, (int32_t)idx)));
                                gstore(B.count + c1, cnt1 + 1);
                                nr = make_double4(R.p1[0], R.p1[1], R.p1[2], pack_meta(0, (int32_t)nl));
                            }
                            j = idx;
                        } else if (is_ins) {
                            const int32_t nl = c0 * cap + cnt0;
                            gstore(B.ent + nl, make_double4(R.p0[0], R.p0[1], R.p0[2], pack_meta(0, (int32_t)N)));
                            gstore(B.count + c0, cnt0 + 1);
                            nr = make_double4(R.p0[0], R.p0[1], R.p0[2], pack_meta(0, (int32_t)nl));
                            j = N;
                        } else if (idx != N - 1) {
                            if (id_last == (int32_t)(N - 1)) rlw = pack_meta(meta_species(rlw), (int32_t)loc);
                            nr = make_double4(rlx, rly, rlz, rlw);
                            gstore_w(B.ent + meta_low(rlw), pack_meta(meta_species(rlw), (int32_t)idx));
                            j = idx;
                        }
                        if (j >= 0) {
                            gstore(B.pos + j, nr);
                            const int64_t t = j - base;
                            if (t >= 0 && t < 2 * W) top[t] = nr;
                        }
                    }
                    // what later moves of this round must not have read
                    if (lane == nmod) {
                        modx = R.c0[0]; mody = R.c0[1]; modz = R.c0[2];
                    }
                    nmod += 1;
                    // a deletion that frees an inner index rewrites the id of particle N-1 in that
                    // particle's cell: that cell counts as modified too (a later removal from it
                    // would otherwise copy the stale id with the cell's last entry)
                    if (type == GCMC_MOVE_DELETE && idx != N - 1 && id_last != (int32_t)(N - 1)) {
                        // its cell from its position (every record lives in the cell of its position)
                        const int32_t rx = spec_axis_cell(rlx, B.invS[0], B.M[0]);
                        const int32_t ry = spec_axis_cell(rly, B.invS[1], B.M[1]);
                        const int32_t rz = spec_axis_cell(rlz, B.invS[2], B.M[2]);
                        if ((rz * B.M[1] + ry) * B.M[0] + rx != (int32_t)c0) {
                            if (lane == nmod) {
                                modx = rx;
                                mody = ry;
                                modz = rz;
                            }
                            nmod += 1;
                        }
                    }
                    if (is_disp && two) {
                        if (lane == nmod) {
                            modx = R.c1[0]; mody = R.c1[1]; modz = R.c1[2];
                        }
                        nmod += 1;
                    }
                    if (lane == ntouch) touched = is_ins ? (int32_t)N : (int32_t)idx;
                    ntouch += 1;
                    if (swap) {
                        if (lane == ntouch) touched = id_last;
                        ntouch += 1;
                    }
                    if (type == GCMC_MOVE_DELETE) {
                        if (lane == ntouch) touched = (int32_t)(N - 1);
                        ntouch += 1;
                    }
                    if (is_disp && two && cnt1 + 1 > maxc) maxc = cnt1 + 1;
                    if (is_ins && cnt0 + 1 > maxc) maxc = cnt0 + 1;
                    okbits |= 1ull << k;
                    N += is_ins ? 1 : (type == GCMC_MOVE_DELETE ? -1 : 0);
                    U += R.dUp;
                    Wvir += R.dWp;
                }
                if (lane == 0) {
                    after_n[k] = N;
                    after_u[k] = U;
                    after_w[k] = Wvir;
                }
                if (nmod > kWave - 2 || ntouch > kWave - 3) {
                    ++k;
                    break;
                }
            }
            // statistics of the k moves decided this round: lane j takes move j (the values
            // lane 0 wrote above, seen by every lane of this wavefront)
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
            {
                const bool mine = lane < k;
                const SpecRec& S = recs[mine ? lane : 0];
                const int t = mine ? S.type : -1;
                const bool a = ((okbits >> lane) & 1) != 0;
                att0 += (double)__builtin_popcountll(__ballot(t == 0));
                att1 += (double)__builtin_popcountll(__ballot(t == 1));
                att2 += (double)__builtin_popcountll(__ballot(t == 2));
                acc0 += (double)__builtin_popcountll(__ballot(a && t == 0));
                acc1 += (double)__builtin_popcountll(__ballot(a && t == 1));
                acc2 += (double)__builtin_popcountll(__ballot(a && t == 2));
                if (mine && !(S.flags & 1)) {
                    stencils += S.two ? 2 : 1;
                    cand += S.cand;
                    evals += S.evals;
                    incut += S.incut;
                }
                if (mine) {
                    const double n = (double)after_n[lane];
                    sum_n += n;
                    sum_n2 += n * n;
                    sum_u += after_u[lane] + tk * n * n;
                    sum_w += after_w[lane];
                }
                // the per-move log, rebuilt from the evaluation, the decision and N after the move
                if (trace && mine) {
                    gcmc_log r;
                    r.type = t;
                    if (S.flags & 1) {
                        r.index = -1; r.accepted = 0; r.flags = 1;
                        r.dU_pair = 0.0; r.dU_tail = 0.0; r.x = r.y = r.z = 0.0; r.arg = 0.0; r.dW_pair = 0.0;
                    } else {
                        const int64_t dn = a ? (t == GCMC_MOVE_INSERT ? 1 : (t == GCMC_MOVE_DELETE ? -1 : 0)) : 0;
                        const int64_t n_before = after_n[lane] - dn;
                        double dUt;
                        r.arg = spec_arg(B, t, S.dUp, n_before, lbase, lpi, lpd, tk, dUt);
                        r.index = t == GCMC_MOVE_INSERT ? (int32_t)n_before : (int32_t)S.idx;
                        r.accepted = a ? 1 : 0;
                        r.flags = 0;
                        r.dU_pair = S.dUp;
                        r.dU_tail = dUt;
                        const bool dsp = t == GCMC_MOVE_DISPLACE;
                        r.x = dsp ? S.p1[0] : S.p0[0];
                        r.y = dsp ? S.p1[1] : S.p0[1];
                        r.z = dsp ? S.p1[2] : S.p0[2];
                        r.dW_pair = S.dWp;
                    }
                    trace[(size_t)bi * n_moves + m + lane] = r;
                }
            }
            if (lane == 0) {
                sh_state[0] = N;
                sh_state[1] = m + k;
                sh_state[2] = err;
                sh_state[3] = err_move;
                sh_u = U;
                sh_w = Wvir;
                sh_maxc = maxc;
                sh_acc[0] = (acc1 + 1.0) / (att1 + 2.0);
                sh_acc[1] = (acc2 + 1.0) / (att2 + 2.0);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();   // commit stores done and visible; the new state published
        N = sh_state[0];
        m = sh_state[1];
        err = (int32_t)sh_state[2];
        err_move = sh_state[3];
        U = sh_u;
        Wvir = sh_w;
        maxc = sh_maxc;
        a_ins = sh_acc[0];
        a_del = sh_acc[1];
    }
    if (wv == 0) {
        for (int off = 32; off >= 1; off >>= 1) {
            stencils += __shfl_xor(stencils, off, kWave);
            cand += __shfl_xor(cand, off, kWave);
            evals += __shfl_xor(evals, off, kWave);
            incut += __shfl_xor(incut, off, kWave);
        }
        sum_n = wave_sum_vec(sum_n);
        sum_n2 = wave_sum_vec(sum_n2);
        sum_u = wave_sum_vec(sum_u);
        sum_w = wave_sum_vec(sum_w);
    }
    if (tid == 0) {
        st->n = N;
        st->u_pair = U;
        st->w_pair = Wvir;
        st->maxcount = maxc;
        st->nsp[0] = N;
        st->counter = (int64_t)(ctr0 + (uint64_t)m);
        if (err != GCMC_OK && st->error == GCMC_OK) {
            st->error = err;
            st->error_move = err_move;
        }
        ChainSums L;
        L.moves = m;
        L.att[0] = (int64_t)att0; L.att[1] = (int64_t)att1; L.att[2] = (int64_t)att2;
        L.acc[0] = (int64_t)acc0; L.acc[1] = (int64_t)acc1; L.acc[2] = (int64_t)acc2;
        L.sum_n = sum_n;
        L.sum_n2 = sum_n2;
        L.sum_u = sum_u;
        L.sum_w = sum_w;
        finish_launch(B, st, L, N, U, Wvir, stencils, cand, evals, incut, stats ? stats + bi : nullptr);
    }
}

using spec_fn = void (*)(const DevBox*, const int32_t*, int64_t, uint64_t, gcmc_stats*, gcmc_log*);

struct SpecCfg {
    int key;   // the waves value of gcmc_box_set_launch that selects it
    int w;
    int ng;    // groups of 64 stencil cells of the microcell path, 0 for the 32-cell path
    spec_fn f;
};

static const SpecCfg kSpecCfgs[] = {
    {2, 2, 0, k_chain_spec<2, 8, 0>},
    {4, 4, 0, k_chain_spec<4, 8, 0>},
    {8, 8, 0, k_chain_spec<8, 8, 0>},
    {16, 16, 0, k_chain_spec<16, 4, 0>},
    {2, 2, kSpecGroupsSmall, k_chain_spec<2, 8, kSpecGroupsSmall>},
    {4, 4, kSpecGroupsSmall, k_chain_spec<4, 8, kSpecGroupsSmall>},
    {8, 8, kSpecGroupsSmall, k_chain_spec<8, 8, kSpecGroupsSmall>},
    {16, 16, kSpecGroupsSmall, k_chain_spec<16, 4, kSpecGroupsSmall>},
    {2, 2, kSpecGroups, k_chain_spec<2, 8, kSpecGroups>},
    {4, 4, kSpecGroups, k_chain_spec<4, 8, kSpecGroups>},
    {8, 8, kSpecGroups, k_chain_spec<8, 8, kSpecGroups>},
    {16, 16, kSpecGroups, k_chain_spec<16, 4, kSpecGroups>},
};

// Groups of 64 cells the box's stencils need: 0 (the 32-cell path) for
// stencils of at most 32 cells whose candidates fit the owner table, else the
// smallest instantiation of the microcell path that holds both stencils of a
// displacement.
static int spec_groups(const DevBox& hb) {
    if (hb.nstencil <= 32 && (int64_t)2 * hb.nstencil * hb.cap <= kSpecOwn) return 0;
    return 2 * hb.nstencil <= kSpecGroupsSmall * kWave ? kSpecGroupsSmall : kSpecGroups;
}

// The speculative kernel handles one species and stencils of at most 512
// cells (32-bit cell slots).
bool spec_supported(const DevBox& hb) {
    return hb.ns == 1 && hb.nstencil <= kSpecMaxStencil && hb.ncells * (int64_t)hb.cap < ((int64_t)1 << 31);
}

bool spec_cfg_exists(int waves) {
    for (const SpecCfg& c : kSpecCfgs)
        if (c.key == waves) return true;
    return false;
}

// A batch launches the path with the most groups any of its boxes needs (the
// microcell path serves any stencil that fits it).
int launch_chain_spec(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                      uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s, int ng) {
    for (const SpecCfg& c : kSpecCfgs) {
        if (c.key == waves && c.ng == ng) {
            hipLaunchKernelGGL(c.f, dim3(n_boxes), dim3(kWave * c.w), 0, s, d_boxes, d_order, n_moves, ctr0, stats,
                               log);
            return 0;
        }
    }
    return -1;
}

int spec_needs_groups(const DevBox& hb) { return spec_groups(hb); }

}  // namespace gcmc
