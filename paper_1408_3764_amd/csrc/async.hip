// Pipelined exact chain: one committer wavefront decides the moves of the
// chain in order while E evaluator wavefronts evaluate the moves ahead of it
// (the same chain as Algorithm 1, move for move).
//
// Evaluator e takes moves e, e + E, e + 2E, ... of the launch.  It starts
// move j once the committer is fewer than AHEAD moves away, reading a
// snapshot of the chain first: the number of decisions whose stores are
// complete (its epoch), the number of decided moves C and the current N.  It
// evaluates j against memory as it finds it (spec_eval: the pick at the N
// expected at j's decision from the C .. j-1 moves' draws), writes the result
// to slot j mod kSlots and marks it ready.
//
// The committer takes move j when its slot is ready.  Memory the evaluation
// read may have been changed by any decision from its epoch on: each decision
// logs the cells it modified and the particle records it rewrote, and the
// evaluation is used only if none of the logged decisions since its epoch
// touched a cell of its stencils or its particle's record, and its pick is
// the one at the current N.  Otherwise the committer makes every earlier store
// complete, publishes that, and asks for the move again (any idle evaluator
// takes it; that evaluation sees the exact state and is always used).  Then
// the move is decided and committed as in the round-based kernel.
//
// Deletions move particle N-1 into the freed index: the committer keeps the
// records of particles mb .. mb + 63 in LDS (mb follows N) together with the
// acceptance prefactors for those N, and updates them with every store.
// Every wait is bounded; a wait that exceeds its bound ends the launch with
// GCMC_ERR_INTERNAL latched in the box.
#include "spec_eval.h"

namespace gcmc {

constexpr int kSlots = 16;        // evaluated moves held ahead of the committer (slot = move mod kSlots)
// AHEAD (template): an evaluator starts a move only this close to the committer
// (at most kSlots - 2).  Farther ahead, the pick at the N expected at the
// decision misses more often.
constexpr int kLogLen = 64;       // decisions kept for validation
constexpr int kWin = 64;          // committer lanes holding particle records mb .. mb + 63

enum { SLOT_FREE = 0, SLOT_READY = 1, SLOT_REDO = 2 };

struct AsyncShared {
    SpecRec rec[kSlots];
    int32_t slot_state[kSlots];
    int32_t slot_move[kSlots];     // move index within the launch
    int32_t slot_epoch[kSlots];    // decisions with complete stores when the evaluation read memory
    int32_t log_cell[kLogLen][3];  // cells a decision modified, x | y << 10 | z << 20; -1 none
    int32_t log_id[kLogLen][3];    // particle indices whose record a decision rewrote; -1 none
    uint64_t cn;                   // (decided moves << 32) | N
    int32_t vis;                   // decisions whose stores are complete
    int32_t redo;                  // a move to evaluate again, -1 none
    int32_t stop;
    int32_t pad;
    double acc[2];                 // running acceptance of insertions, deletions
    // the committer's window: records of particles mb .. mb + 63, prefactors at N = mb + t
    double4 wrec[kWin];
    double wlpi[kWin], wlpd[kWin];
};

__device__ __forceinline__ int32_t lds_load(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t lds_load64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Publish a flag after this wavefront's earlier LDS accesses.  The fence is
// limited to LDS: a workgroup-scope release of all memory would first wait for
// every outstanding global store (the committer's stores of the move just
// decided), which only the store-visibility counter needs.
__device__ __forceinline__ void lds_publish(int32_t* p, int32_t v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_publish64(uint64_t* p, uint64_t v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Publish the store-visibility counter: every global store issued before it is complete.
__device__ __forceinline__ void publish_visible(int32_t* p, int32_t v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int32_t pack_cell(int32_t x, int32_t y, int32_t z) { return x | (y << 10) | (z << 20); }

// Does logged cell `pc` (packed) lie in the stencil of centre c?
__device__ __forceinline__ bool logged_in_stencil(const DevBox& B, int32_t pc, const int32_t* c) {
    return pc >= 0 && in_stencil(B, pc & 0x3FF, (pc >> 10) & 0x3FF, pc >> 20, c);
}

// Fill the window with particles mb .. mb + 63 (one lane each): `from` holds
// the old window's records for lanes whose index it covered (shift = new mb - old mb).
__device__ __forceinline__ void window_fill(const DevBox& B, AsyncShared& S, int64_t mb, int64_t old_mb, int64_t N,
                                            int lane) {
    const int64_t j = mb + lane;
    const int64_t o = j - old_mb;   // lane of the old window that held particle j
    double4 nr = make_double4(0, 0, 0, 0);
    if (old_mb >= 0 && o >= 0 && o < kWin) nr = S.wrec[o];
    else if (j < N) nr = gload(B.pos + j);
    const double n = (double)j;
    const double lpi = log(B.V / (B.lambda3 * (n + 1.0)));
    const double lpd = j >= 1 ? log((B.lambda3 * n) / B.V) : 0.0;
    // every lane has read the old window before any lane writes the new one
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    S.wrec[lane] = nr;
    S.wlpi[lane] = lpi;
    S.wlpd[lane] = lpd;
    // wait for the loads here: loads and stores share one counter, and a load still
    // pending in the decision loop would make later waits wait for its stores too
    __builtin_amdgcn_s_waitcnt(0);
}

template <int E, int CR, int AHEAD>
__global__ __launch_bounds__(kWave*(E + 1)) void k_chain_async(const DevBox* __restrict__ boxes,
                                                                const int32_t* __restrict__ order, int64_t n_moves,
                                                                uint64_t ctr0, gcmc_stats* stats, gcmc_log* trace) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ int32_t offs[64];
    __shared__ uint8_t own[E][kSpecOwn];
    __shared__ double pq[E][kPairRing];   // each evaluator's queue of in-cutoff pairs
    __shared__ AsyncShared S;
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;
    const DevBox B = hot_copy(boxes[blockIdx.x]);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    BoxState* st = B.st;
    if (ctr0 == GCMC_COUNTER_CONTINUE) ctr0 = (uint64_t)st->counter;
    const int64_t N0 = uni64(st->n);
    const int32_t err0 = uni(st->error);
    const bool no_full = !(B.full[0] | B.full[1] | B.full[2]);
    const int32_t spin_cap = wait_bound(B.wait_limit);   // polls of a bounded wait
    for (int t = tid; t < B.nstencil; t += blockDim.x) {
        const uint32_t pk = gload(B.stab + t);
        const int tx = pk & 0x3FF, ty = (pk >> 10) & 0x3FF, tz = pk >> 20;
        tab[t] = pk;
        if (t < 64) offs[t] = ((tz - B.k[2]) * B.M[1] + (ty - B.k[1])) * B.M[0] + (tx - B.k[0]);
    }
    for (int t = tid; t < kSlots; t += blockDim.x) {
        S.slot_state[t] = SLOT_FREE;
        S.slot_move[t] = -1;
    }
    if (tid == 0) {
        S.cn = (uint64_t)(uint32_t)N0;
        S.vis = 0;
        S.redo = -1;
        S.stop = (err0 != GCMC_OK || B.ns != 1 || n_moves <= 0) ? 1 : 0;
        S.acc[0] = 0.5;
        S.acc[1] = 0.5;
    }
    __syncthreads();

    if (wv != 0) {
        // ================================================== evaluator
        const int e = wv - 1;
        int32_t jn = e;
        int32_t spins = 0;
        while (true) {
            if (uni(lds_load(&S.stop))) break;
            int32_t target = -1;
            const int32_t r = uni(lds_load(&S.redo));
            if (r >= 0) {
                int32_t won = 0;
                if (lane == 0) {
                    int32_t expect = r;
                    won = __hip_atomic_compare_exchange_strong(&S.redo, &expect, -1, __ATOMIC_ACQ_REL,
                                                               __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)
                              ? 1
                              : 0;
                }
                if (__builtin_amdgcn_readlane(won, 0)) target = r;
            }
            if (target < 0) {
                const int32_t C = uni((int32_t)(lds_load64(&S.cn) >> 32));
                if (jn >= n_moves || jn - C >= AHEAD) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > spin_cap) {
                        if (lane == 0) lds_publish(&S.stop, 1);
                        break;
                    }
                    continue;
                }
                target = jn;
                jn += E;
            }
            spins = 0;
            // snapshot: complete decisions first, then the decided count and N
            const int32_t vis = uni(lds_load(&S.vis));
            const uint64_t cn = lds_load64(&S.cn);
            const int32_t C = uni((int32_t)(cn >> 32));
            const int64_t N = uni64((int64_t)(uint32_t)cn);
            const double a_ins = unid(S.acc[0]), a_del = unid(S.acc[1]);
            const int s = target % kSlots;
            SpecKey key;
            spec_eval<CR, 0, 0>(B, tab, offs, own[e], pq[e], nullptr, ctr0 + (uint64_t)C, target - C, N, no_full, a_ins,
                                a_del, &S.rec[s], key);
            if (lane == 0) {
                S.slot_move[s] = target;
                S.slot_epoch[s] = vis;
                lds_publish(&S.slot_state[s], SLOT_READY);
            }
        }
        return;
    }

    // ====================================================== committer
    // the committer is the chain's critical path: it issues before the evaluators sharing its SIMD
    __builtin_amdgcn_s_setprio(3);
    int64_t N = N0;
    double U = unid(st->u_pair);
    double Wvir = unid(st->w_pair);
    int32_t maxc = uni(st->maxcount);
    int32_t err = err0;
    int64_t err_move = uni64(st->error_move);
    if (err == GCMC_OK && B.ns != 1) {
        err = GCMC_ERR_UNSUPPORTED;
        err_move = (int64_t)ctr0;
    }
    const double tk = B.tailK[0];
    const int cap = B.cap;
    int64_t att0 = 0, att1 = 0, att2 = 0, acc0 = 0, acc1 = 0, acc2 = 0;
    double sum_n = 0.0, sum_u = 0.0, sum_n2 = 0.0, sum_w = 0.0;
    int64_t stencils = 0, cand = 0, evals = 0, incut = 0;
    int64_t mb = N - 32 > 0 ? N - 32 : 0;
    window_fill(B, S, mb, -1, N, lane);
    int32_t vis_pub = 0;
    int64_t j = 0;
    for (; err == GCMC_OK && j < n_moves; ++j) {
        // keep N - 1 and N inside the window
        if ((N - mb < 8 && mb > 0) || N - mb > kWin - 8) {
            // the new window's particles below the old one come from memory: the
            // committer's stores to them must be complete first
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            const int64_t nb = (N - mb < 8) ? (mb - 32 > 0 ? mb - 32 : 0) : mb + 32;
            window_fill(B, S, nb, mb, N, lane);
            mb = nb;
        }
        const int s = (int)(j % kSlots);
        // ---- the evaluation of move j
        int32_t spins = 0;
        while (!(uni(lds_load(&S.slot_state[s])) == SLOT_READY && uni(S.slot_move[s]) == (int32_t)j)) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin_cap) break;
        }
        if (spins > spin_cap) {
            err = GCMC_ERR_INTERNAL;
            err_move = (int64_t)(ctr0 + (uint64_t)j);
            break;
        }
        const uint64_t ctr = ctr0 + (uint64_t)j;
        bool retried = false;
        int type = 0;
        for (;;) {
            const SpecRec& R = S.rec[s];
            type = __builtin_amdgcn_readfirstlane(R.type);
            if (type != GCMC_MOVE_INSERT && N == 0) break;   // empty box: rejected without an evaluation
            bool valid = !(R.flags & 1);
            if (type != GCMC_MOVE_INSERT) valid = valid && spec_pick(R.u2, R.u7, N) == R.idx;
            // decisions since the evaluation's epoch that may have changed what it read
            const int32_t ep = uni(S.slot_epoch[s]);
            const int32_t nd = (int32_t)j - ep;
            valid = valid && nd <= kLogLen;
            if (valid && nd > 0) {
                int32_t cc[3] = {R.c0[0], R.c0[1], R.c0[2]};
                int32_t cn[3] = {R.c1[0], R.c1[1], R.c1[2]};
                bool hit = false;
                if (lane < nd) {
                    const int q = (ep + lane) % kLogLen;
                    const int32_t idx = (int32_t)R.idx;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const int32_t pc = S.log_cell[q][a];
                        hit = hit || logged_in_stencil(B, pc, cc) ||
                              (type == GCMC_MOVE_DISPLACE && logged_in_stencil(B, pc, cn));
                        hit = hit || (type != GCMC_MOVE_INSERT && S.log_id[q][a] == idx);
                    }
                }
                valid = __ballot(hit) == 0;
            }
            if (uni(valid ? 1 : 0)) break;
            if (retried) {   // an evaluation on the exact state is always valid
                err = GCMC_ERR_INTERNAL;
                break;
            }
            // evaluate again on the exact state: make every earlier store complete, publish it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            vis_pub = (int32_t)j;
            if (lane == 0) {
                publish_visible(&S.vis, vis_pub);
                lds_publish(&S.slot_state[s], SLOT_REDO);
                lds_publish(&S.redo, (int32_t)j);
            }
            spins = 0;
            while (!(uni(lds_load(&S.slot_state[s])) == SLOT_READY)) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > spin_cap) break;
            }
            if (spins > spin_cap) {
                err = GCMC_ERR_INTERNAL;
                break;
            }
            retried = true;
        }
        if (err != GCMC_OK) {
            err_move = (int64_t)ctr;
            break;
        }
        const SpecRec R = S.rec[s];   // the whole record in one batch of LDS reads
        // the decision's log entry: nothing modified until shown otherwise
        int32_t lc0 = -1, lc1 = -1, lc2 = -1, li0 = -1, li1 = -1, li2 = -1;
        if (type != GCMC_MOVE_INSERT && N == 0) {
            att0 += type == 0; att1 += type == 1; att2 += type == 2;
            if (trace && lane == 0) {
                gcmc_log r;
                r.type = type; r.index = -1; r.accepted = 0; r.flags = 1;
                r.dU_pair = 0.0; r.dU_tail = 0.0; r.x = r.y = r.z = 0.0; r.arg = 0.0; r.dW_pair = 0.0;
                trace[(size_t)bi * n_moves + j] = r;
            }
            sum_u += U;
            sum_w += Wvir;
        } else {
            const int64_t idx = R.idx;
            const bool is_disp = type == GCMC_MOVE_DISPLACE, is_ins = type == GCMC_MOVE_INSERT;
            const double dUp = R.dUp;
            const double dUt = is_disp ? 0.0 : tk * (is_ins ? (2.0 * (double)N + 1.0) : (1.0 - 2.0 * (double)N));
            const double dU = dUp + dUt;
            const int wl = (int)(N - mb);
            const double lpref = is_disp ? 0.0 : (is_ins ? S.wlpi[wl] : S.wlpd[wl]);
            const double arg = is_disp ? -(B.beta * dU)
                                       : (is_ins ? lpref + B.beta * (B.mu - dU) : lpref - B.beta * (B.mu + dU));
            const bool ok = __builtin_amdgcn_readfirstlane((dU == dU && R.lnA < arg) ? 1 : 0) != 0;
            const int two = R.two;
            const int32_t cnt0 = R.cnt0, cnt1 = R.cnt1;
            const int64_t n_old = N;
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
                const int64_t loc = meta_low(R.rec.w);
                const int64_t c0 = R.cl0, c1 = R.cl1;
                const bool removes = (type == GCMC_MOVE_DELETE) || (is_disp && two);
                const int64_t last = c0 * cap + cnt0 - 1;
                const bool swap = removes && loc != last;
                const int32_t id_last = swap ? meta_low(R.elast.w) : -1;
                // the record of particle N-1 as of now
                double4 rl = make_double4(0.0, 0.0, 0.0, 0.0);
                if (type == GCMC_MOVE_DELETE) {
                    rl = S.wrec[N - 1 - mb];
                }
                if (swap) {
                    const double w = pack_meta(meta_species(R.elast.w), (int32_t)loc);
                    if (lane == 0) {
                        gstore(B.ent + loc, R.elast);
                        gstore_w(B.pos + id_last, w);
                    }
                    const int64_t t = (int64_t)id_last - mb;
                    if (lane == 0 && t >= 0 && t < kWin) S.wrec[t].w = w;
                }
                if (removes && lane == 0) gstore(B.count + c0, cnt0 - 1);
                double4 nr = make_double4(0.0, 0.0, 0.0, 0.0);
                int64_t jp = -1;
                if (is_disp) {
                    if (!two) {
                        if (lane == 0) gstore(B.ent + loc, make_double4(R.p1[0], R.p1[1], R.p1[2], pack_meta(0, (int32_t)idx)));
                        nr = make_double4(R.p1[0], R.p1[1], R.p1[2], R.rec.w);
                    } else {
                        const int64_t nl = c1 * cap + cnt1;
                        if (lane == 0) {
                            gstore(B.ent + nl, make_double4(R.p1[0], R.p1[1], R.p1[2], pack_meta(0, (int32_t)idx)));
                            gstore(B.count + c1, cnt1 + 1);
                        }
                        nr = make_double4(R.p1[0], R.p1[1], R.p1[2], pack_meta(0, (int32_t)nl));
                    }
                    jp = idx;
                } else if (is_ins) {
                    const int64_t nl = c0 * cap + cnt0;
                    if (lane == 0) {
                        gstore(B.ent + nl, make_double4(R.p0[0], R.p0[1], R.p0[2], pack_meta(0, (int32_t)N)));
                        gstore(B.count + c0, cnt0 + 1);
                    }
                    nr = make_double4(R.p0[0], R.p0[1], R.p0[2], pack_meta(0, (int32_t)nl));
                    jp = N;
                } else if (idx != N - 1) {
                    if (id_last == (int32_t)(N - 1)) rl.w = pack_meta(meta_species(rl.w), (int32_t)loc);
                    nr = rl;
                    if (lane == 0) gstore_w(B.ent + meta_low(rl.w), pack_meta(meta_species(rl.w), (int32_t)idx));
                    jp = idx;
                }
                if (jp >= 0) {
                    if (lane == 0) gstore(B.pos + jp, nr);
                    const int64_t t = jp - mb;
                    if (lane == 0 && t >= 0 && t < kWin) S.wrec[t] = nr;
                }
                // the log entry: cells modified, particle records rewritten
                lc0 = pack_cell(R.c0[0], R.c0[1], R.c0[2]);
                if (is_disp && two) lc1 = pack_cell(R.c1[0], R.c1[1], R.c1[2]);
                if (type == GCMC_MOVE_DELETE && idx != N - 1 && id_last != (int32_t)(N - 1)) {
                    // the relabelled particle's cell, from its position (every record lives in the
                    // cell of its position)
                    const int32_t rx = spec_axis_cell(rl.x, B.invS[0], B.M[0]);
                    const int32_t ry = spec_axis_cell(rl.y, B.invS[1], B.M[1]);
                    const int32_t rz = spec_axis_cell(rl.z, B.invS[2], B.M[2]);
                    if ((rz * B.M[1] + ry) * B.M[0] + rx != (int32_t)c0) lc2 = pack_cell(rx, ry, rz);
                }
                li0 = is_ins ? (int32_t)N : (int32_t)idx;
                li1 = swap ? id_last : -1;
                li2 = (type == GCMC_MOVE_DELETE) ? (int32_t)(N - 1) : -1;
                if (is_disp && two && cnt1 + 1 > maxc) maxc = cnt1 + 1;
                if (is_ins && cnt0 + 1 > maxc) maxc = cnt0 + 1;
                acc0 += type == 0; acc1 += type == 1; acc2 += type == 2;
                N += is_ins ? 1 : (type == GCMC_MOVE_DELETE ? -1 : 0);
                U += dUp;
                Wvir += R.dWp;
            }
            att0 += type == 0; att1 += type == 1; att2 += type == 2;
            stencils += two ? 2 : 1;
            cand += R.cand;
            evals += R.evals;
            incut += R.incut;
            if (trace && lane == 0) {
                gcmc_log r;
                r.type = type;
                r.index = is_ins ? (int32_t)n_old : (int32_t)idx;
                r.accepted = ok ? 1 : 0;
                r.flags = 0;
                r.dU_pair = dUp;
                r.dU_tail = dUt;
                r.x = is_disp ? R.p1[0] : R.p0[0];
                r.y = is_disp ? R.p1[1] : R.p0[1];
                r.z = is_disp ? R.p1[2] : R.p0[2];
                r.arg = arg;
                r.dW_pair = R.dWp;
                trace[(size_t)bi * n_moves + j] = r;
            }
            sum_n += (double)N;
            sum_n2 += (double)N * (double)N;
            sum_u += U + tk * (double)N * (double)N;
            sum_w += Wvir;
        }
        // publish the decision: its log entry, the free slot, the decided count and N
        if (lane == 0) {
            const int q = (int)(j % kLogLen);
            S.log_cell[q][0] = lc0; S.log_cell[q][1] = lc1; S.log_cell[q][2] = lc2;
            S.log_id[q][0] = li0; S.log_id[q][1] = li1; S.log_id[q][2] = li2;
            lds_publish(&S.slot_state[s], SLOT_FREE);
            lds_publish64(&S.cn, ((uint64_t)(j + 1) << 32) | (uint64_t)(uint32_t)N);
        }
        // completed stores are published now and then (and always before asking for a move again)
        const int s1 = (int)((j + 1) % kSlots);
        const bool next_ready = uni(lds_load(&S.slot_state[s1])) == SLOT_READY && uni(S.slot_move[s1]) == (int32_t)(j + 1);
        if ((int32_t)(j + 1) - vis_pub >= 8 || !next_ready) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            vis_pub = (int32_t)(j + 1);
            if (lane == 0) {
                S.acc[0] = ((double)acc1 + 1.0) / ((double)att1 + 2.0);
                S.acc[1] = ((double)acc2 + 1.0) / ((double)att2 + 2.0);
                publish_visible(&S.vis, vis_pub);
            }
        }
    }
    if (lane == 0) lds_publish(&S.stop, 1);
    if (lane == 0) {
        st->n = N;
        st->u_pair = U;
        st->w_pair = Wvir;
        st->maxcount = maxc;
        st->nsp[0] = N;
        st->counter = (int64_t)(ctr0 + (uint64_t)j);
        if (err != GCMC_OK && st->error == GCMC_OK) {
            st->error = err;
            st->error_move = err_move;
        }
        ChainSums L;
        L.moves = j;
        L.att[0] = att0; L.att[1] = att1; L.att[2] = att2;
        L.acc[0] = acc0; L.acc[1] = acc1; L.acc[2] = acc2;
        L.sum_n = sum_n;
        L.sum_n2 = sum_n2;
        L.sum_u = sum_u;
        L.sum_w = sum_w;
        finish_launch(B, st, L, N, U, Wvir, stencils, cand, evals, incut, stats ? stats + bi : nullptr);
    }
}

using async_fn = void (*)(const DevBox*, const int32_t*, int64_t, uint64_t, gcmc_stats*, gcmc_log*);

struct AsyncCfg {
    int key;     // the waves value of gcmc_box_set_launch that selects it
    int waves;   // evaluators + the committer
    async_fn f;
};

static const AsyncCfg kAsyncCfgs[] = {
    {4, 4, k_chain_async<3, 8, 4>},
    {8, 8, k_chain_async<7, 8, 4>},
};

// Cells are logged packed in 10 bits per axis.
// The pipelined kernel evaluates with the 32-cell path of the speculative
// evaluation only.
bool async_supported(const DevBox& hb) {
    return hb.ns == 1 && hb.nstencil <= 32 && (int64_t)2 * hb.nstencil * hb.cap <= kSpecOwn &&
           hb.ncells * (int64_t)hb.cap < ((int64_t)1 << 31) && hb.M[0] <= 1024 && hb.M[1] <= 1024 &&
           hb.M[2] <= 1024;
}

bool async_cfg_exists(int waves) {
    for (const AsyncCfg& c : kAsyncCfgs)
        if (c.key == waves) return true;
    return false;
}

int launch_chain_async(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                       uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s) {
    if (n_moves >= ((int64_t)1 << 31)) return -1;
    for (const AsyncCfg& c : kAsyncCfgs) {
        if (c.key == waves) {
            hipLaunchKernelGGL(c.f, dim3(n_boxes), dim3(kWave * c.waves), 0, s, d_boxes, d_order, n_moves, ctr0,
                               stats, log);
            return 0;
        }
    }
    return -1;
}

}  // namespace gcmc
