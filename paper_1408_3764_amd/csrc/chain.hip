// The persistent Markov-chain kernel: one workgroup advances one box through
// many moves of Algorithm 1 in a single launch (the paper's multi-move kernel,
// Sec. 3.3.4), with device-side Philox draws and Metropolis tests.
//
// On one compute unit a move is bound by vector-instruction issue and by the
// latency of its memory round trips, so the kernel keeps both small:
//  * slot decomposition (stencil cell, entry, which position) of every lane's
//    rows is computed once per occupancy level, with the linear offset of the
//    stencil cell from the centre cell; for a centre cell away from the box
//    faces a candidate's address is one add and one multiply-add;
//  * the counters and 32-byte entries of all slots are loaded in one round
//    trip; while it is in flight the next move's draws are computed (one
//    Philox block per lane, four lanes) and the record of the particle it will
//    pick is loaded, and ln A and the log prefactor of this move are formed;
//  * each wavefront compacts its valid candidates (k below the cell's count,
//    not the moving particle) into LDS and evaluates only those;
//  * the centre cells' counters and the old cell's last entry come back with
//    the gather, so the commit (Sec. 3.2.5: swap-with-last removal, append) is
//    stores only; prefetched records are validated after it.
// Wave-uniform decisions go through readfirstlane so they never sit in
// exec-masked code.  The chain is exactly the sequential one.
#include "trial.h"

namespace gcmc {

struct Head {
    U8 u;
    int type;
    int64_t idx;       // picked particle, -1 for insertion or empty box
    double4 rec;       // pos[idx]
    double4 rlast;     // pos[N-1] (deletion: the particle that takes idx)
};

__device__ __forceinline__ int move_type(const DevBox& B, const U8& u) {
    return (u.u[0] < B.p_disp) ? GCMC_MOVE_DISPLACE : ((u.u[1] < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
}

__device__ __forceinline__ int64_t pick_index(const U8& u, int64_t n) { return pick_particle(u.u[2], u.u[7], n); }

// Draws, type and pick of move ctr for N = n; issues the record loads.
__device__ __forceinline__ void head_of(const DevBox& B, uint64_t ctr, int64_t n, Head& H) {
    H.u = move_uniforms_lanes(B.seed, ctr, B.box_id);
    H.type = __builtin_amdgcn_readfirstlane(move_type(B, H.u));
    H.idx = -1;
    if (H.type != GCMC_MOVE_INSERT && n > 0) {
        H.idx = pick_index(H.u, n);
        H.rec = gload(B.pos + H.idx);
        if (H.type == GCMC_MOVE_DELETE) H.rlast = gload(B.pos + (n - 1));
    }
}

// Cell of position w of the trial, made wave-uniform (the positions are the
// same in every lane; saying so keeps the stencil arithmetic scalar).
__device__ __forceinline__ void locate_uniform(const DevBox& B, Trial& T, int w) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
        T.c[w][a] = __builtin_amdgcn_readfirstlane(axis_cell(T.p[w][a], B.invS[a], B.M[a]));
    T.cl[w] = ((int64_t)T.c[w][2] * B.M[1] + T.c[w][1]) * B.M[0] + T.c[w][0];
}

__device__ __forceinline__ bool interior(const DevBox& B, const int32_t* c) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) ok = ok && c[a] >= B.k[a] && c[a] <= B.M[a] - 1 - B.k[a];
    return ok;
}

// Packed per-row slot description: k | which << 21 | valid << 22.
constexpr int kSlotW = 21, kSlotV = 22;

template <int W, int R>
__global__ __launch_bounds__(kWave* W) void k_chain(const DevBox* __restrict__ boxes,
                                                     const int32_t* __restrict__ order, int64_t n_moves,
                                                     uint64_t ctr0, gcmc_stats* stats, gcmc_log* trace) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ double red[2][4 * W];
    __shared__ int32_t sh_cnt[2][2];     // counters of the two centre cells, per buffer
    __shared__ double4 sh_last[2];       // last entry of the old centre cell, per buffer
    __shared__ int64_t wred[3][W];
    __shared__ double4 cbuf[W][kWave * R];   // per-wavefront compacted candidates
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;
    const DevBox B = hot_copy(boxes[blockIdx.x]);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    double4* my = cbuf[wv];
    BoxState* st = B.st;

    if (ctr0 == GCMC_COUNTER_CONTINUE) ctr0 = (uint64_t)st->counter;
    int64_t N = st->n;
    double U = st->u_pair;
    double Wvir = st->w_pair;
    int32_t maxc = st->maxcount;
    int32_t err = st->error;
    int64_t err_move = st->error_move;
    int64_t att[3] = {0, 0, 0}, acc_n[3] = {0, 0, 0};
    double sum_n = 0.0, sum_u = 0.0, sum_n2 = 0.0, sum_w = 0.0;
    const double tk = B.tailK[0];
    const int cap = B.cap;
    const int M0 = B.M[0], M01 = B.M[0] * B.M[1];
    const bool no_full = !(B.full[0] | B.full[1] | B.full[2]);
    int64_t m = 0;
    int ev = 0;
    int64_t stencils = 0;
    Work wk;
    load_stencil(B, tab);
    __syncthreads();

    // per-lane slot table for the current occupancy level
    int lg_cached = -1;
    bool fast_ok = false;
    int32_t sk[R], soff[R];

    if (err == GCMC_OK && B.ns != 1) {
        err = GCMC_ERR_UNSUPPORTED;
        err_move = (int64_t)ctr0;
    }
    if (err == GCMC_OK && n_moves > 0) {
        Head H;
        head_of(B, ctr0, N, H);
        for (; m < n_moves; ++m) {
            const uint64_t ctr = ctr0 + (uint64_t)m;
            att[H.type] += 1;
            // ---------------------------------------------------- empty box
            if (H.type != GCMC_MOVE_INSERT && N == 0) {
                if (trace && tid == 0) {
                    gcmc_log r;
                    r.type = H.type; r.index = -1; r.accepted = 0; r.flags = 1;
                    r.dU_pair = 0.0; r.dU_tail = 0.0; r.x = r.y = r.z = 0.0; r.arg = 0.0; r.dW_pair = 0.0;
                    trace[(size_t)bi * n_moves + m] = r;
                }
                sum_u += U;
                sum_w += Wvir;
                if (m + 1 < n_moves) head_of(B, ctr + 1, N, H);
                continue;
            }
            // ------------------------------------------------------ trial
            Trial T;
            T.type = H.type;
            T.sp = 0;
            T.idx = H.idx;
            if (H.type == GCMC_MOVE_INSERT) {
                T.npos = 1;
                T.same = 0;
                T.meta = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) T.p[0][a] = wrap_into_box(B.L[a] * H.u.u[4 + a], B.L[a]);
                locate_uniform(B, T, 0);
            } else {
                T.meta = H.rec.w;
                T.p[0][0] = H.rec.x; T.p[0][1] = H.rec.y; T.p[0][2] = H.rec.z;
                locate_uniform(B, T, 0);
                if (H.type == GCMC_MOVE_DISPLACE) {
                    T.npos = 2;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        T.p[1][a] = wrap_into_box(T.p[0][a] + B.max_disp * (2.0 * H.u.u[4 + a] - 1.0), B.L[a]);
                    locate_uniform(B, T, 1);
                    T.same = __builtin_amdgcn_readfirstlane(T.cl[0] == T.cl[1] ? 1 : 0);
                } else {
                    T.npos = 1;
                    T.same = 0;
                }
            }
            const int lg = __builtin_amdgcn_readfirstlane(log2_ceil(maxc));
            const int NS = B.nstencil << lg;
            const int two = (T.npos == 2 && !T.same) ? 1 : 0;
            const int total = NS << two;
            const int gmask = (1 << lg) - 1;
            if (lg != lg_cached) {
                // slot table of this occupancy level (both stencils' ranges)
                lg_cached = lg;
                fast_ok = no_full && (2 * NS <= kWave * W * R) && lg <= 10;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int s = r * kWave * W + tid;
                    const int w = s >= NS ? 1 : 0;
                    const int q = s - w * NS;
                    const int t = (s < 2 * NS) ? (q >> lg) : 0;
                    const int k = q & gmask;
                    const uint32_t pk = tab[t];
                    const int dx = (int)(pk & 0x3FF) - B.k[0];
                    const int dy = (int)((pk >> 10) & 0x3FF) - B.k[1];
                    const int dz = (int)(pk >> 20) - B.k[2];
                    soff[r] = dz * M01 + dy * M0 + dx;
                    sk[r] = (k & 0x3FF) | (w << kSlotW) | ((s < 2 * NS ? 1 : 0) << kSlotV);
                }
            }
            const bool fast = __builtin_amdgcn_readfirstlane(
                                  (fast_ok && interior(B, T.c[0]) && (!two || interior(B, T.c[1]))) ? 1 : 0) != 0;
            const int buf = ev & 1;
            const int32_t excl = (int32_t)T.idx;
            const int32_t cl0 = (int32_t)T.cl[0], cl1 = (int32_t)T.cl[1];
            double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
            Head Hn;
            bool have_next = false;
            double lnA = 0.0, lpref = 0.0;
            // -------------------------------------- gather + evaluate passes
            for (int base = 0; base < total; base += kWave * W * R) {
                double4 e[R];
                int32_t cnt[R], kk[R], cc[R], which[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    int32_t c;
                    bool in;
                    int k, w;
                    if (fast) {
                        const int32_t pk = sk[r];
                        w = (pk >> kSlotW) & 1;
                        in = ((pk >> kSlotV) & 1) && (two || !w);
                        k = pk & 0x3FF;
                        c = (w ? cl1 : cl0) + soff[r];
                    } else {
                        const int s = base + r * kWave * W + tid;
                        in = s < total;
                        w = (two && s >= NS) ? 1 : 0;
                        const int q = in ? s - w * NS : 0;
                        const int t = q >> lg;
                        k = q & gmask;
                        const int32_t cx = w ? T.c[1][0] : T.c[0][0];
                        const int32_t cy = w ? T.c[1][1] : T.c[0][1];
                        const int32_t cz = w ? T.c[1][2] : T.c[0][2];
                        c = (int32_t)stencil_cell(B, tab[t], cx, cy, cz);
                    }
                    if (!in) c = cl0;
                    const int kc = k < cap ? k : cap - 1;
                    cnt[r] = in ? gload(B.count + c) : 0;
                    e[r] = gload(B.ent + ((size_t)(uint32_t)c * (uint32_t)cap + kc));
                    kk[r] = k;
                    cc[r] = in ? c : -1;
                    which[r] = w;
                }
                if (!have_next) {
                    // overlaps the gather: this move's ln A and log prefactor, the next
                    // move's draws and record (N assumed unchanged)
                    lnA = log(H.u.u[3]);
                    if (T.type == GCMC_MOVE_INSERT) lpref = log(B.V / (B.lambda3 * (double)(N + 1)));
                    else if (T.type == GCMC_MOVE_DELETE) lpref = log((B.lambda3 * (double)N) / B.V);
                    if (m + 1 < n_moves) head_of(B, ctr + 1, N, Hn);
                    have_next = true;
                }
                // centre records, then compaction of the valid candidates of this wavefront
                int nv = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // the centre cell appears once in a stencil: found by its index
                    if (cc[r] == (which[r] ? cl1 : cl0)) {
                        if (kk[r] == 0) sh_cnt[buf][which[r]] = cnt[r];
                        if (which[r] == 0 && kk[r] == cnt[r] - 1) sh_last[buf] = e[r];
                    }
                    const bool valid = kk[r] < cnt[r] && meta_low(e[r].w) != excl;
                    const uint64_t bal = __ballot(valid);
                    if (valid) {
                        const int at = nv + __popcll(bal & ((1ull << lane) - 1ull));
                        my[at] = make_double4(e[r].x, e[r].y, e[r].z, (double)which[r]);
                    }
                    nv += __popcll(bal);
                }
                __builtin_amdgcn_wave_barrier();
                wk.cand += (lane == 0) ? nv : 0;
                for (int j = lane; j < nv; j += kWave) {
                    const double4 c4 = my[j];
                    if (T.npos == 1) {
                        sa += pair_uw<false>(B, T.p[0], 0, c4, wk.incut, wa);
                        wk.evals += 1;
                    } else if (!two) {
                        sa += pair_uw<false>(B, T.p[0], 0, c4, wk.incut, wa);
                        sb += pair_uw<false>(B, T.p[1], 0, c4, wk.incut, wb);
                        wk.evals += 2;
                    } else if (c4.w != 0.0) {
                        sb += pair_uw<false>(B, T.p[1], 0, c4, wk.incut, wb);
                        wk.evals += 1;
                    } else {
                        sa += pair_uw<false>(B, T.p[0], 0, c4, wk.incut, wa);
                        wk.evals += 1;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
            ++ev;
            stencils += two ? 2 : 1;
            // ----------------------------------------------------- reduce
            double ea = wave_sum_uniform(sa);
            double eb = (T.npos == 2) ? wave_sum_uniform(sb) : 0.0;
            double va = wave_sum_uniform(wa);
            double vb = (T.npos == 2) ? wave_sum_uniform(wb) : 0.0;
            if (W > 1) {
                if (lane == 0) {
                    red[buf][4 * wv] = ea;
                    red[buf][4 * wv + 1] = eb;
                    red[buf][4 * wv + 2] = va;
                    red[buf][4 * wv + 3] = vb;
                }
                __syncthreads();
                double ta = 0.0, tb = 0.0, ua = 0.0, ub = 0.0;
#pragma unroll
                for (int v = 0; v < W; ++v) {
                    ta += red[buf][4 * v];
                    tb += red[buf][4 * v + 1];
                    ua += red[buf][4 * v + 2];
                    ub += red[buf][4 * v + 3];
                }
                ea = ta;
                eb = tb;
                va = ua;
                vb = ub;
            }
            // ----------------------------------------------------- decide
            // Accept iff ln A < ln(ratio) (Eqs. 3-5); the same test as A < min(1, ratio).
            const bool is_disp = T.type == GCMC_MOVE_DISPLACE, is_ins = T.type == GCMC_MOVE_INSERT;
            const double dUp = is_disp ? (eb - ea) : (is_ins ? ea : -ea);
            const double dWp = is_disp ? (vb - va) : (is_ins ? va : -va);
            const double dUt = is_disp ? 0.0 : tk * (is_ins ? (2.0 * (double)N + 1.0) : (1.0 - 2.0 * (double)N));
            const double dU = dUp + dUt;
            const double arg = is_disp ? -(B.beta * dU)
                                       : (is_ins ? lpref + B.beta * (B.mu - dU) : lpref - B.beta * (B.mu + dU));
            const bool ok = __builtin_amdgcn_readfirstlane((dU == dU && lnA < arg) ? 1 : 0) != 0;
            // ----------------------------------------------------- commit
            const int64_t n_old = N;
            int64_t touched0 = -1, touched1 = -1;
            if (ok) {
                if (W == 1) __syncthreads();   // LDS records of this wave visible to lane 0
                const int32_t cnt0 = __builtin_amdgcn_readfirstlane(sh_cnt[buf][0]);
                const int32_t cnt1 = two ? __builtin_amdgcn_readfirstlane(sh_cnt[buf][1]) : 0;
                const double4 elast = sh_last[buf];
                int e = GCMC_OK;
                if (T.type == GCMC_MOVE_INSERT) {
                    if (N >= B.max_n) e = GCMC_ERR_CAPACITY;
                    else if (cnt0 >= cap) e = GCMC_ERR_CELL_OVERFLOW;
                } else if (T.type == GCMC_MOVE_DISPLACE && two) {
                    if (cnt1 >= cap) e = GCMC_ERR_CELL_OVERFLOW;
                }
                if (e != GCMC_OK) {
                    err = e;
                    err_move = (int64_t)ctr;
                    att[T.type] -= 1;
                    break;
                }
                const int64_t loc = meta_low(T.meta);
                const int64_t c0 = T.cl[0], c1 = T.cl[1];
                // swap-with-last removal from the old cell (displacement across cells, deletion)
                const bool removes = (T.type == GCMC_MOVE_DELETE) || (T.type == GCMC_MOVE_DISPLACE && two);
                const int64_t last = c0 * cap + cnt0 - 1;
                const bool swap = removes && loc != last;
                const int32_t id_last = swap ? meta_low(elast.w) : -1;
                if (tid == 0) {
                    if (swap) {
                        gstore(B.ent + loc, elast);
                        gstore_w(B.pos + id_last, pack_meta(meta_species(elast.w), (int32_t)loc));
                    }
                    if (removes) gstore(B.count + c0, cnt0 - 1);
                    if (T.type == GCMC_MOVE_DISPLACE) {
                        if (!two) {
                            gstore(B.ent + loc, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], pack_meta(0, (int32_t)T.idx)));
                            gstore(B.pos + T.idx, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], T.meta));
                        } else {
                            const int64_t nl = c1 * cap + cnt1;
                            gstore(B.ent + nl, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], pack_meta(0, (int32_t)T.idx)));
                            gstore(B.count + c1, cnt1 + 1);
                            gstore(B.pos + T.idx, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], pack_meta(0, (int32_t)nl)));
                        }
                    } else if (T.type == GCMC_MOVE_INSERT) {
                        const int64_t nl = c0 * cap + cnt0;
                        gstore(B.ent + nl, make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(0, (int32_t)N)));
                        gstore(B.count + c0, cnt0 + 1);
                        gstore(B.pos + N, make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(0, (int32_t)nl)));
                    } else if (T.idx != N - 1) {
                        // particle N-1 takes index idx
                        double4 r = H.rlast;
                        if (id_last == (int32_t)(N - 1)) r.w = pack_meta(meta_species(r.w), (int32_t)loc);
                        gstore(B.pos + T.idx, r);
                        gstore_w(B.ent + (meta_low(r.w)), pack_meta(meta_species(r.w), (int32_t)T.idx));
                    }
                }
                if (T.type == GCMC_MOVE_DISPLACE && two && cnt1 + 1 > maxc) maxc = cnt1 + 1;
                if (T.type == GCMC_MOVE_INSERT && cnt0 + 1 > maxc) maxc = cnt0 + 1;
                touched0 = (T.type == GCMC_MOVE_INSERT) ? N : T.idx;
                touched1 = id_last;
                acc_n[T.type] += 1;
                N += (T.type == GCMC_MOVE_INSERT) ? 1 : ((T.type == GCMC_MOVE_DELETE) ? -1 : 0);
                U += dUp;
                Wvir += dWp;
                __syncthreads();   // commit stores complete and visible to the workgroup
            }
            if (trace && tid == 0) {
                gcmc_log r;
                r.type = T.type;
                r.index = (T.type == GCMC_MOVE_INSERT) ? (int32_t)n_old : (int32_t)T.idx;
                r.accepted = ok ? 1 : 0;
                r.flags = 0;
                r.dU_pair = dUp;
                r.dU_tail = dUt;
                const int w = (T.type == GCMC_MOVE_DISPLACE) ? 1 : 0;
                r.x = T.p[w][0]; r.y = T.p[w][1]; r.z = T.p[w][2];
                r.arg = arg;
                r.dW_pair = dWp;
                trace[(size_t)bi * n_moves + m] = r;
            }
            sum_n += (double)N;
            sum_n2 += (double)N * (double)N;
            sum_u += U + tk * (double)N * (double)N;
            sum_w += Wvir;
            // ------------------------------------- validate the prefetch
            if (m + 1 < n_moves) {
                if (Hn.type != GCMC_MOVE_INSERT && N > 0) {
                    const int64_t i2 = pick_index(Hn.u, N);
                    if (N != n_old || Hn.idx < 0 || i2 != Hn.idx || i2 == touched0 || i2 == touched1) {
                        Hn.idx = i2;
                        Hn.rec = gload(B.pos + i2);
                    }
                    if (Hn.type == GCMC_MOVE_DELETE &&
                        (N != n_old || N - 1 == touched0 || N - 1 == touched1))
                        Hn.rlast = gload(B.pos + (N - 1));
                } else {
                    Hn.idx = -1;
                }
                H = Hn;
            }
        }
    }
    // launch-wide work counters
    {
        int64_t c = wk.cand, e = wk.evals, q = wk.incut;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            c += __shfl_xor(c, off, kWave);
            e += __shfl_xor(e, off, kWave);
            q += __shfl_xor(q, off, kWave);
        }
        __syncthreads();
        if (lane == 0) {
            wred[0][wv] = c;
            wred[1][wv] = e;
            wred[2][wv] = q;
        }
        __syncthreads();
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
        for (int t = 0; t < 3; ++t) {
            L.att[t] = att[t];
            L.acc[t] = acc_n[t];
        }
        L.sum_n = sum_n;
        L.sum_n2 = sum_n2;
        L.sum_u = sum_u;
        L.sum_w = sum_w;
        int64_t c = 0, e = 0, q = 0;
        for (int v = 0; v < W; ++v) {
            c += wred[0][v];
            e += wred[1][v];
            q += wred[2][v];
        }
        finish_launch(B, st, L, N, U, Wvir, stencils, c, e, q, stats ? stats + bi : nullptr);
    }
}

using chain_fn = void (*)(const DevBox*, const int32_t*, int64_t, uint64_t, gcmc_stats*, gcmc_log*);

struct ChainCfg {
    int w, r;
    chain_fn f;
};

static const ChainCfg kChainCfgs[] = {
    {1, 8, k_chain<1, 8>}, {2, 8, k_chain<2, 8>}, {4, 2, k_chain<4, 2>}, {4, 4, k_chain<4, 4>},
    {4, 8, k_chain<4, 8>}, {8, 2, k_chain<8, 2>}, {8, 4, k_chain<8, 4>},
};

int launch_chain(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int rows, int64_t n_moves,
                 uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s) {
    for (const ChainCfg& c : kChainCfgs) {
        if (c.w == waves && c.r == rows) {
            hipLaunchKernelGGL(c.f, dim3(n_boxes), dim3(kWave * c.w), 0, s, d_boxes, d_order, n_moves, ctr0, stats,
                               log);
            return 0;
        }
    }
    return -1;
}

bool chain_cfg_exists(int waves, int rows) {
    for (const ChainCfg& c : kChainCfgs)
        if (c.w == waves && c.r == rows) return true;
    return false;
}

}  // namespace gcmc
