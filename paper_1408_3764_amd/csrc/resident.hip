// The persistent chain of Algorithm 1 for a small box held in local memory.
//
// In a box of a few hundred to a couple of thousand particles the 27-cell
// stencil covers most or all of the box, so the cell list prunes little, every
// accepted move makes the rest of a speculative round of the global-memory
// kernels stale, and a move costs a chain of dependent memory round trips of
// about a microsecond each.  Here one workgroup copies the box's coordinates
// into LDS once per launch and runs every move against that copy.
//
// Rounds of W moves: wavefront w evaluates move m + w against every other
// particle of the state at the start of the round (the energy of a move is the
// sum over all particles inside the cutoff, Eq. 1 with the strict cutoff: the
// same pairs the cell list finds), and wavefront 0 decides the moves in order.
// A move whose particle an earlier accepted move of the round changed, or
// whose pick at the current N is another particle, ends the round and is
// evaluated again in the next.  Every other move is used with its energy and
// virial corrected for the earlier accepted moves of the round: removing a
// particle at a and adding one at b changes the move's sums by f(b) - f(a),
// f(r) the pair terms of r with the move's new position minus those with its
// old one, so a few pair terms, one lane per earlier move, replace a new pass
// over the box.  The accepted moves are written to the LDS copy in order after
// the round.  Particles with an index of kResCap or more (a box that grows past
// it) are read from and written to global memory instead: correct, slower.
//
// The cells are not maintained during the launch.  At its end the workgroup
// writes the coordinates back and rebuilds the box's cell list in the layout
// of gcmc_cell_build (entries of a cell in particle-id order, back-pointers in
// the records), so every other kernel and call finds the box as it expects.
#include "spec_eval.h"

namespace gcmc {

constexpr int kResCap = 2048;   // particles whose coordinates live in LDS
constexpr int kResRing = 64;    // moves prepared at once

// What a move needs from its draws, prepared for kResRing moves at a time:
// the type, ln A, the 53 bits of the pick fields as an integer, the floor
// fallback's uniform, and the displacement (or the inserted position).
struct ResMove {
    int32_t type;
    uint32_t klo, khi;
    double u2, lnA;
    double q[3];
};

// One move's evaluation against the round's starting state.
struct ResRec {
    int32_t type, flags;        // flags bit 0: displacement or deletion in an empty box
    int64_t idx;                // picked particle (-1 for an insertion)
    double pold[3], pnew[3];    // old position (displacement, deletion), new (displacement, insertion)
    double dUp, dWp;            // pair energy and pair virial change against the round's start
    int32_t cand, evals, incut, pad;
};

// An accepted move of the round: it removed a particle at a (displacement,
// deletion) and added one at b (displacement, insertion); N before it.
struct ResMod {
    int32_t type, pad;
    int64_t idx, n_before;
    double a[3], b[3];
};

// The particle a displacement or deletion picks among n >= 1, on wave-uniform
// integers: the rule of pick_particle with the spare draw's 53 bits given as
// an integer.
__device__ __forceinline__ int64_t res_pick(const ResMove& r, int64_t n) {
    if (n <= 1) return 0;
    const uint64_t k = ((uint64_t)(uint32_t)uni((int32_t)r.khi) << 32) | (uint32_t)uni((int32_t)r.klo);
    const int b = 64 - __clzll((long long)(n - 1));
    const uint64_t mask = (1ull << b) - 1ull;
    for (int sh = 53 - b; sh >= 0; sh -= b) {
        const uint64_t v = (k >> sh) & mask;
        if (v < (uint64_t)n) return (int64_t)v;
    }
    const int64_t i = (int64_t)floor(r.u2 * (double)n);
    return uni64(i > n - 1 ? n - 1 : i);
}

// The same pick with every lane on its own move.
__device__ __forceinline__ int64_t res_pick_lane(const ResMove& r, int64_t n) {
    if (n <= 1) return 0;
    const uint64_t k = ((uint64_t)r.khi << 32) | (uint64_t)r.klo;
    const int b = 64 - __clzll((long long)(n - 1));
    const uint64_t mask = (1ull << b) - 1ull;
    int64_t idx = -1;
    for (int sh = 53 - b; sh >= 0 && idx < 0; sh -= b) {
        const uint64_t v = (k >> sh) & mask;
        if (v < (uint64_t)n) idx = (int64_t)v;
    }
    if (idx < 0) {
        const int64_t i = (int64_t)floor(r.u2 * (double)n);
        idx = i > n - 1 ? n - 1 : i;
    }
    return idx;
}

template <int W>
__global__ __launch_bounds__(kWave* W) void k_chain_resident(const DevBox* __restrict__ boxes,
                                                              const int32_t* __restrict__ order, int64_t n_moves,
                                                              uint64_t ctr0, gcmc_stats* stats, gcmc_log* trace) {
    __shared__ double px[kResCap], py[kResCap], pz[kResCap];
    __shared__ DrawRing<kResRing> dring;
    __shared__ ResMove mv[kResRing];
    // log acceptance prefactors for N = lbase + t: insertion V / (Lambda^3 (N + 1)), deletion
    // Lambda^3 N / V (the moves prepared together change N by at most one each)
    __shared__ double lpi[2 * kResRing + 1], lpd[2 * kResRing + 1];
    __shared__ ResRec rec[W];
    __shared__ ResMod mods[W];
    __shared__ double pq[W][kPairRing];   // each wavefront's queue of in-cutoff pairs
    // corr[k][j]: the change of move k's pair energy and virial if move j < k of the round is
    // accepted (move j's removed and added positions against move k's positions)
    __shared__ double corr_e[W][W], corr_w[W][W];
    __shared__ int32_t ready[W];          // round whose evaluation wavefront w has published
    __shared__ int64_t sh_n, sh_k, sh_nacc, sh_err, sh_err_move;
    __shared__ double sh_u, sh_w;
    __shared__ int64_t wred[4][W];
    __shared__ int32_t sh_flag;
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
    int32_t err = st->error;
    int64_t err_move = st->error_move;
    const double tk = B.tailK[0];
    const double rc2 = B.rc2, eps4 = B.eps4[0], sig2 = B.sig2[0];
    const int32_t spin_cap = wait_bound(B.wait_limit);
    // statistics, kept by wavefront 0
    int64_t att0 = 0, att1 = 0, att2 = 0, acc0 = 0, acc1 = 0, acc2 = 0;
    double sum_n = 0.0, sum_u = 0.0, sum_n2 = 0.0, sum_w = 0.0;
    int64_t cand = 0, evals = 0, incut = 0;

    auto get = [&](int64_t j) -> double3 {
        if (j < kResCap) return make_double3(px[j], py[j], pz[j]);
        return gload_xyz(B.pos + j);
    };
    auto put = [&](int64_t j, const double* q) {
        if (j < kResCap) {
            px[j] = q[0];
            py[j] = q[1];
            pz[j] = q[2];
        } else {
            gstore(B.pos + j, make_double4(q[0], q[1], q[2], 0.0));
        }
    };
    // energy and virial of one pair inside the cutoff, added to (e, v); pairs outside add zero
    auto pair = [&](double r2, double& e, double& v, int32_t& nin) {
        const bool in = r2 < rc2;
        nin += in ? 1 : 0;
        double w = 0.0;
        const double u = lj_uw_from_r2(in ? r2 : rc2, rc2, eps4, sig2, w);
        e += in ? u : 0.0;
        v += in ? w : 0.0;
    };

    {
        const int64_t nl = N < kResCap ? N : kResCap;
        for (int64_t j = tid; j < nl; j += blockDim.x) {
            const double4 r = gload(B.pos + j);
            px[j] = r.x;
            py[j] = r.y;
            pz[j] = r.z;
        }
    }
    if (tid == 0) sh_flag = 0;
    if (tid < W) ready[tid] = -1;
    if (err == GCMC_OK && B.ns != 1) {
        err = GCMC_ERR_UNSUPPORTED;
        err_move = (int64_t)ctr0;
    }
    __syncthreads();
    int64_t m = 0;
    int64_t prep_end = 0;   // moves m' < prep_end have their draws prepared (with the tables)
    int64_t lbase = 0;
    int32_t rnd = 0;
    while (err == GCMC_OK && m < n_moves) {
        rnd = rnd == INT32_MAX ? 1 : rnd + 1;
        if (m + W > prep_end) {
            // moves m .. m + kResRing - 1: Philox block t & 3 of move m + t / 4 per thread, the
            // prefactor tables for every N those moves can meet, then one thread per move derives
            // what the move needs
            const uint64_t ctr = ctr0 + (uint64_t)m;
            for (int t = tid; t < 4 * kResRing; t += blockDim.x)
                draw_block(B, &dring, ctr + (uint64_t)(t >> 2), t & 3);
            lbase = N - kResRing;
            for (int t = tid; t < 2 * (2 * kResRing + 1); t += blockDim.x) {
                const bool del = t > 2 * kResRing;
                const int64_t n = lbase + (del ? t - (2 * kResRing + 1) : t);
                if (n >= 0) {
                    const double x = del ? (B.lambda3 * (double)n) / B.V : B.V / (B.lambda3 * (double)(n + 1));
                    if (del) lpd[t - (2 * kResRing + 1)] = log(x);
                    else lpi[t] = log(x);
                }
            }
            __syncthreads();
            if (tid < kResRing) {
                const int sl = (int)((ctr + (uint64_t)tid) & (uint64_t)(kResRing - 1));
                ResMove r;
                r.type = dring.type[sl];
                const uint64_t k = (uint64_t)(dring.u7[sl] * 9007199254740992.0);
                r.klo = (uint32_t)k;
                r.khi = (uint32_t)(k >> 32);
                r.u2 = dring.u2[sl];
                r.lnA = dring.lnA[sl];
                const double ud[3] = {dring.px[sl], dring.py[sl], dring.pz[sl]};
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    r.q[a] = r.type == GCMC_MOVE_INSERT ? wrap_into_box(B.L[a] * ud[a], B.L[a])
                                                        : B.max_disp * (2.0 * ud[a] - 1.0);
                mv[sl] = r;
            }
            prep_end = m + kResRing;
            __syncthreads();
        }
        const int kend = (n_moves - m) < W ? (int)(n_moves - m) : W;
        // ------------------------------------------------ evaluate move m + wv
        if (wv < kend) {
            const int s = (int)((ctr0 + (uint64_t)(m + wv)) & (uint64_t)(kResRing - 1));
            const ResMove& R = mv[s];
            const int type = uni(R.type);
            ResRec out;
            out.type = type;
            out.flags = 0;
            out.idx = -1;
            out.dUp = out.dWp = 0.0;
            out.cand = out.evals = out.incut = out.pad = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) out.pold[a] = out.pnew[a] = 0.0;
            if (type != GCMC_MOVE_INSERT && N == 0) {
                out.flags = 1;
            } else {
                const bool disp = type == GCMC_MOVE_DISPLACE, ins = type == GCMC_MOVE_INSERT;
                double p0[3], p1[3] = {0.0, 0.0, 0.0};
                int64_t idx = -1;
                if (ins) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) p0[a] = R.q[a];
                } else {
                    idx = res_pick(R, N);
                    const double3 o = get(idx);
                    p0[0] = o.x; p0[1] = o.y; p0[2] = o.z;
                    if (disp) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) p1[a] = wrap_into_box(p0[a] + R.q[a], B.L[a]);
                    }
                }
                double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
                uint32_t qhead = 0, qtail = 0;
                int32_t n_eval = 0, n_c = 0;
                int64_t n_in = 0;
                for (int64_t j0 = 0; j0 < N; j0 += kWave) {
                    const int64_t j = j0 + lane;
                    const bool valid = j < N && j != idx;
                    const double3 e = valid ? get(j) : make_double3(0.0, 0.0, 0.0);
                    n_c += valid ? 1 : 0;
                    spec_pair_queue(B, type, 0, valid, false, p0, p1, e, true, pq[wv], qhead, qtail, sa, sb, wa, wb,
                                    n_eval, n_in);
                }
                if (qtail != qhead) pair_drain(B, pq[wv], qhead, qtail - qhead, sa, sb, wa, wb);
                // lane j < wv: the correction if the earlier move j of the round is accepted, from the
                // positions move j takes (its pick at the round's N, its draws)
                {
                    double ce = 0.0, cw = 0.0;
                    if (lane < wv) {
                        const ResMove& Rj = mv[(int)((ctr0 + (uint64_t)(m + lane)) & (uint64_t)(kResRing - 1))];
                        const int tj = Rj.type;
                        if (tj == GCMC_MOVE_INSERT || N > 0) {
                            double aj[3] = {0.0, 0.0, 0.0}, bj[3] = {0.0, 0.0, 0.0};
                            if (tj == GCMC_MOVE_INSERT) {
#pragma unroll
                                for (int a = 0; a < 3; ++a) bj[a] = Rj.q[a];
                            } else {
                                const double3 o = get(res_pick_lane(Rj, N));
                                aj[0] = o.x; aj[1] = o.y; aj[2] = o.z;
                                if (tj == GCMC_MOVE_DISPLACE) {
#pragma unroll
                                    for (int a = 0; a < 3; ++a) bj[a] = wrap_into_box(aj[a] + Rj.q[a], B.L[a]);
                                }
                            }
                            // f(r): pair terms with this move's new position minus those with its old one
                            int32_t dummy = 0;
                            double enb = 0.0, wnb = 0.0, eob = 0.0, wob = 0.0, ena = 0.0, wna = 0.0, eoa = 0.0, woa = 0.0;
                            const double* pn = disp ? p1 : p0;
                            const double3 ja = make_double3(aj[0], aj[1], aj[2]), jb = make_double3(bj[0], bj[1], bj[2]);
                            if (tj != GCMC_MOVE_DELETE) {
                                if (!(type == GCMC_MOVE_DELETE)) pair(spec_dist2(B, pn, jb, true), enb, wnb, dummy);
                                if (!ins) pair(spec_dist2(B, p0, jb, true), eob, wob, dummy);
                            }
                            if (tj != GCMC_MOVE_INSERT) {
                                if (!(type == GCMC_MOVE_DELETE)) pair(spec_dist2(B, pn, ja, true), ena, wna, dummy);
                                if (!ins) pair(spec_dist2(B, p0, ja, true), eoa, woa, dummy);
                            }
                            ce = (enb - eob) - (ena - eoa);
                            cw = (wnb - wob) - (wna - woa);
                        }
                        corr_e[wv][lane] = ce;
                        corr_w[wv][lane] = cw;
                    }
                }
                sa = wave_sum_uniform(sa);
                sb = wave_sum_uniform(sb);
                wa = wave_sum_uniform(wa);
                wb = wave_sum_uniform(wb);
                n_c = wave_sum_i32_uniform(n_c);
                n_eval = wave_sum_i32_uniform(n_eval);
                const int32_t n_inc = wave_sum_i32_uniform((int32_t)n_in);
                out.idx = idx;
                out.dUp = disp ? (sb - sa) : (ins ? sa : -sa);
                out.dWp = disp ? (wb - wa) : (ins ? wa : -wa);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    out.pold[a] = ins ? 0.0 : p0[a];
                    out.pnew[a] = disp ? p1[a] : (ins ? p0[a] : 0.0);
                }
                out.cand = n_c;
                out.evals = n_eval;
                out.incut = n_inc;
            }
            if (lane == 0) rec[wv] = out;
            if (wv == 0) {
                // its own record, read by every lane of this wavefront below
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
            } else {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                if (lane == 0) __hip_atomic_store(&ready[wv], rnd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        // ------------------------------------------------ decide in order (wavefront 0)
        if (wv == 0) {
            int64_t Nc = N;
            double Uc = U, Wc = Wvir;
            int nacc = 0;
            int32_t ntouch = 0;
            int64_t touched = -1;   // lane t < ntouch: a particle index an accepted move changed
            uint64_t accbits = 0;   // bit j: move j of the round accepted
            int k = 0;
            for (; k < kend; ++k) {
                const uint64_t ctr = ctr0 + (uint64_t)(m + k);
                if (k > 0) {
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
                const ResRec& R = rec[k];
                const int type = uni(R.type);
                const int s = (int)(ctr & (uint64_t)(kResRing - 1));
                if (R.flags & 1) {
                    // the empty-box rejection holds only while the box is still empty
                    if (Nc != 0) break;
                    if (type == GCMC_MOVE_DISPLACE) att0 += 1;
                    else att2 += 1;
                    sum_u += Uc;
                    sum_w += Wc;
                    if (trace && lane == 0) {
                        gcmc_log r;
                        r.type = type; r.index = -1; r.accepted = 0; r.flags = 1;
                        r.dU_pair = 0.0; r.dU_tail = 0.0; r.x = r.y = r.z = 0.0; r.arg = 0.0; r.dW_pair = 0.0;
                        trace[(size_t)bi * n_moves + (m + k)] = r;
                    }
                    continue;
                }
                const bool disp = type == GCMC_MOVE_DISPLACE, ins = type == GCMC_MOVE_INSERT;
                const int64_t idx = uni64(R.idx);
                if (!ins) {
                    if (res_pick(mv[s], Nc) != idx) break;
                    if (__ballot(lane < ntouch && touched == idx) != 0) break;
                }
                // corrections for the accepted earlier moves of this round (prepared by this move's
                // wavefront, one lane each), summed over the lanes in a fixed order
                double cE = 0.0, cW = 0.0;
                if (accbits != 0) {
                    const bool use = lane < k && ((accbits >> lane) & 1ull) != 0;
                    cE = wave_sum_uniform(use ? corr_e[k][lane] : 0.0);
                    cW = wave_sum_uniform(use ? corr_w[k][lane] : 0.0);
                }
                const double dUp = R.dUp + cE;
                const double dWp = R.dWp + cW;
                // ---- decide at the current N (Eqs. 3-5)
                const double dUt = disp ? 0.0 : tk * (ins ? (2.0 * (double)Nc + 1.0) : (1.0 - 2.0 * (double)Nc));
                const double dU = dUp + dUt;
                const double lpref = disp ? 0.0 : (ins ? lpi[Nc - lbase] : lpd[Nc - lbase]);
                const double arg = disp ? -(B.beta * dU)
                                        : (ins ? lpref + B.beta * (B.mu - dU) : lpref - B.beta * (B.mu + dU));
                const bool ok = __builtin_amdgcn_readfirstlane((dU == dU && mv[s].lnA < arg) ? 1 : 0) != 0;
                if (ok && ins && Nc >= B.max_n) {
                    err = GCMC_ERR_CAPACITY;
                    err_move = (int64_t)ctr;
                    break;
                }
                if (disp) att0 += 1;
                else if (ins) att1 += 1;
                else att2 += 1;
                // work counters of the decided moves, kept by lane 0 (the lanes are summed at the end)
                if (lane == 0) {
                    cand += R.cand;
                    evals += R.evals;
                    incut += R.incut;
                }
                const int64_t n_old = Nc;
                if (ok) {
                    if (lane == 0) {
                        ResMod& J = mods[nacc];
                        J.type = type;
                        J.pad = 0;
                        J.idx = ins ? Nc : idx;
                        J.n_before = Nc;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            J.a[a] = R.pold[a];
                            J.b[a] = R.pnew[a];
                        }
                    }
                    // the indices whose particle changed: the moved or deleted one, the inserted
                    // one, and the last one a deletion relabels
                    if (lane == ntouch) touched = ins ? Nc : idx;
                    ntouch += 1;
                    if (type == GCMC_MOVE_DELETE) {
                        if (lane == ntouch) touched = Nc - 1;
                        ntouch += 1;
                    }
                    nacc += 1;
                    accbits |= 1ull << k;
                    if (disp) acc0 += 1;
                    else if (ins) acc1 += 1;
                    else acc2 += 1;
                    Nc += ins ? 1 : (disp ? 0 : -1);
                    Uc += dUp;
                    Wc += dWp;
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
                }
                if (trace && lane == 0) {
                    gcmc_log r;
                    r.type = type;
                    r.index = ins ? (int32_t)n_old : (int32_t)idx;
                    r.accepted = ok ? 1 : 0;
                    r.flags = 0;
                    r.dU_pair = dUp;
                    r.dU_tail = dUt;
                    r.x = R.pnew[0]; r.y = R.pnew[1]; r.z = R.pnew[2];
                    if (type == GCMC_MOVE_DELETE) {
                        r.x = R.pold[0]; r.y = R.pold[1]; r.z = R.pold[2];
                    }
                    r.arg = arg;
                    r.dW_pair = dWp;
                    trace[(size_t)bi * n_moves + (m + k)] = r;
                }
                sum_n += (double)Nc;
                sum_n2 += (double)Nc * (double)Nc;
                sum_u += Uc + tk * (double)Nc * (double)Nc;
                sum_w += Wc;
            }
            if (lane == 0) {
                sh_n = Nc;
                sh_u = Uc;
                sh_w = Wc;
                sh_k = k;
                sh_nacc = nacc;
                sh_err = err;
                sh_err_move = err_move;
            }
        }
        __syncthreads();   // every evaluation read the round's state; the decisions published
        const int64_t nacc = sh_nacc;
        if (tid == 0) {
            // the accepted moves into the LDS copy, in order
            for (int j = 0; j < (int)nacc; ++j) {
                const ResMod& J = mods[j];
                if (J.type == GCMC_MOVE_DELETE) {
                    if (J.idx != J.n_before - 1) {
                        const double3 l = get(J.n_before - 1);
                        const double q[3] = {l.x, l.y, l.z};
                        put(J.idx, q);
                    }
                } else {
                    put(J.idx, J.b);
                }
            }
        }
        N = sh_n;
        U = sh_u;
        Wvir = sh_w;
        err = (int32_t)sh_err;
        err_move = sh_err_move;
        m += sh_k;
        __syncthreads();   // the new state visible to every wavefront
    }
    // ---------------------------------------------------- coordinates back, cells rebuilt
    // (after any move; a launch that ran none changed nothing)
    __syncthreads();
    const int64_t n_cells = m > 0 ? B.ncells : 0;
    const int64_t n_bin = m > 0 ? N : 0;
    for (int64_t c = tid; c < n_cells; c += blockDim.x) gstore(B.count + c, 0);
    __syncthreads();
    const int cap = B.cap;
    bool over = false;
    for (int64_t j = tid; j < n_bin; j += blockDim.x) {
        const double3 p = get(j);
        // every coordinate goes back, also a particle whose cell overflows (its back-pointer
        // is set with its slot below)
        gstore(B.pos + j, make_double4(p.x, p.y, p.z, 0.0));
        const int64_t c = cell_of_point(B, p.x, p.y, p.z);
        const int32_t k = atomicAdd(&B.count[c], 1);
        if (k < cap) gstore(B.ent + (c * cap + k), make_double4(p.x, p.y, p.z, pack_meta(0, (int32_t)j)));
        else over = true;
    }
    if (over) atomicOr(&sh_flag, 1);
    __syncthreads();
    int32_t maxc = 0;
    if (cap <= kWave) {
        // one wavefront per cell: an entry's slot is the number of the cell's entries with a smaller id
        for (int64_t c = wv; c < n_cells; c += W) {
            // the counters were raised by other wavefronts' atomics: read them where those happened
            int32_t cnt = __hip_atomic_load(B.count + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cnt = __builtin_amdgcn_readfirstlane(cnt > cap ? cap : cnt);
            if (cnt == 0) continue;
            double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
            int32_t id = INT32_MAX;
            if (lane < cnt) {
                v = gload(B.ent + (c * cap + lane));
                id = meta_low(v.w);
            }
            int32_t rank = 0;
            for (int q = 0; q < cnt; ++q) rank += (__builtin_amdgcn_readlane(id, q) < id) ? 1 : 0;
            if (lane < cnt) {
                const int32_t slot = (int32_t)(c * cap + rank);
                gstore(B.ent + slot, v);
                gstore(B.pos + id, make_double4(v.x, v.y, v.z, pack_meta(0, slot)));
            }
            maxc = cnt > maxc ? cnt : maxc;
        }
    } else {
        for (int64_t c = tid; c < n_cells; c += blockDim.x) {
            int32_t cnt = __hip_atomic_load(B.count + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cnt > cap) cnt = cap;
            double4* e = B.ent + c * cap;
            for (int32_t a = 1; a < cnt; ++a) {
                const double4 v = e[a];
                const int32_t id = meta_low(v.w);
                int32_t b = a - 1;
                while (b >= 0 && meta_low(e[b].w) > id) {
                    e[b + 1] = e[b];
                    --b;
                }
                e[b + 1] = v;
            }
            for (int32_t a = 0; a < cnt; ++a) {
                const double4 v = e[a];
                gstore(B.pos + meta_low(v.w), make_double4(v.x, v.y, v.z, pack_meta(0, (int32_t)(c * cap + a))));
            }
            maxc = cnt > maxc ? cnt : maxc;
        }
    }
    maxc = wave_max_i32_uniform(maxc);
    {
        int64_t c = cand, e = evals, q = incut;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            c += __shfl_xor(c, off, kWave);
            e += __shfl_xor(e, off, kWave);
            q += __shfl_xor(q, off, kWave);
        }
        if (lane == 0) {
            wred[0][wv] = c;
            wred[1][wv] = e;
            wred[2][wv] = q;
            wred[3][wv] = maxc;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int64_t c = 0, e = 0, q = 0, mx = 0;
        for (int v = 0; v < W; ++v) {
            c += wred[0][v];
            e += wred[1][v];
            q += wred[2][v];
            mx = wred[3][v] > mx ? wred[3][v] : mx;
        }
        if (err == GCMC_OK && sh_flag) {
            // a cell of the rebuilt list overflowed: the chain itself is complete; a rebuild with a
            // larger capacity (gcmc_cell_build) restores the cells and clears the error
            err = GCMC_ERR_CELL_OVERFLOW;
            err_move = (int64_t)(ctr0 + (uint64_t)m);
        }
        st->n = N;
        st->u_pair = U;
        st->w_pair = Wvir;
        st->maxcount = (int32_t)mx > st->maxcount ? (int32_t)mx : st->maxcount;
        st->nsp[0] = N;
        st->counter = (int64_t)(ctr0 + (uint64_t)m);
        if (err != GCMC_OK && st->error == GCMC_OK) {
            st->error = err;
            st->error_move = err_move;
        }
        ChainSums L;
        L.moves = m;
        L.att[0] = att0; L.att[1] = att1; L.att[2] = att2;
        L.acc[0] = acc0; L.acc[1] = acc1; L.acc[2] = acc2;
        L.sum_n = sum_n;
        L.sum_n2 = sum_n2;
        L.sum_u = sum_u;
        L.sum_w = sum_w;
        finish_launch(B, st, L, N, U, Wvir, 0, c, e, q, stats ? stats + bi : nullptr);
    }
}

using resident_fn = void (*)(const DevBox*, const int32_t*, int64_t, uint64_t, gcmc_stats*, gcmc_log*);

bool resident_cfg_exists(int waves) { return waves == 4 || waves == 8; }

int launch_chain_resident(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                          uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s) {
    resident_fn f = waves == 4 ? k_chain_resident<4> : (waves == 8 ? k_chain_resident<8> : nullptr);
    if (!f) return -1;
    hipLaunchKernelGGL(f, dim3(n_boxes), dim3(kWave * waves), 0, s, d_boxes, d_order, n_moves, ctr0, stats, log);
    return 0;
}

}  // namespace gcmc
