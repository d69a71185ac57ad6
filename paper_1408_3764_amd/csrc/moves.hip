// Trial-move energy evaluation over the cell stencil, the incremental cell
// update on acceptance, and the persistent Markov-chain kernel.
//
// Mapping (gfx950, wave64).  One workgroup of W wavefronts evaluates one move.
// The stencil of a position is its cell plus the cells within k cells of it
// (Sec. 3.2: the 27 adjoining cells for S >= rc).  Every stencil cell owns G
// consecutive "slots", G = the power of two at or above the largest cell
// count, and slot q of the move is handled by lane q mod (64 W): lane loads
// the cell's counter and its entry k = q mod G in the same instruction
// group, so one memory round trip brings all candidates of the move
// (coordinates and id, 32 bytes, cell-major) into registers; slots with k at
// or past the count are masked.  A displacement whose old and new positions
// share a cell evaluates both positions against the same candidates (the
// reuse of Sec. 3.2.4); otherwise the two stencils occupy two slot ranges.
// Per-lane sums are reduced across the wavefront with cross-lane shuffles and
// across wavefronts through LDS, in a fixed order.
#include "gcmc_internal.h"

namespace gcmc {

struct Trial {
    int type;
    int npos;          // positions evaluated: 1 (insert/delete) or 2 (displace)
    int same;          // displacement inside one cell
    int sp;            // species of the moving / inserted particle
    int64_t idx;       // particle index (displace/delete), -1 for insertion
    double meta;       // pos[idx].w
    double p[2][3];    // p[0] old / insertion / deleted position, p[1] new position
    int32_t c[2][3];   // their cell coordinates
    int64_t cl[2];     // their linear cells
};

__device__ __forceinline__ void locate(const DevBox& B, Trial& T, int w) {
#pragma unroll
    for (int a = 0; a < 3; ++a) T.c[w][a] = axis_cell(T.p[w][a], B.invS[a], B.M[a]);
    T.cl[w] = ((int64_t)T.c[w][2] * B.M[1] + T.c[w][1]) * B.M[0] + T.c[w][0];
}

// Stencil offsets (packed tx | ty << 10 | tz << 20) into LDS.
__device__ __forceinline__ void build_stencil(const DevBox& B, uint32_t* tab) {
    const int sx = B.span[0], sy = B.span[1];
    for (int t = threadIdx.x; t < B.nstencil; t += blockDim.x) {
        const int tx = t % sx, ty = (t / sx) % sy, tz = t / (sx * sy);
        tab[t] = (uint32_t)tx | ((uint32_t)ty << 10) | ((uint32_t)tz << 20);
    }
}

__device__ __forceinline__ int log2_ceil(int v) {
    return v <= 1 ? 0 : 32 - __clz(v - 1);
}

template <bool MIX>
__device__ __forceinline__ double pair_energy(const DevBox& B, const double* p, int sp, const double4& e) {
    const double r2 = dist2(B, p[0], p[1], p[2], e.x, e.y, e.z);
    if (MIX) {
        const int q = sp * B.ns + meta_species(e.w);
        return lj_from_r2(r2, B.rc2, B.eps4[q], B.sig2[q]);
    }
    return lj_from_r2(r2, B.rc2, B.eps4[0], B.sig2[0]);
}

// Block-wide: ea = sum over candidates of u(p[0], .), eb = sum of u(p[1], .)
// (eb only for displacements).  `red` holds 2*W doubles of LDS.
// Per-lane work counters, summed over a whole launch.
struct Work {
    int64_t cand = 0;   // candidate records read (valid slots)
    int64_t evals = 0;  // pair distances evaluated
    int64_t incut = 0;  // pairs inside the cutoff
};

template <bool MIX>
__device__ __forceinline__ double pair_energy_w(const DevBox& B, const double* p, int sp, const double4& e,
                                                int64_t& incut) {
    const double r2 = dist2(B, p[0], p[1], p[2], e.x, e.y, e.z);
    incut += (r2 < B.rc2) ? 1 : 0;
    if (MIX) {
        const int q = sp * B.ns + meta_species(e.w);
        return lj_from_r2(r2, B.rc2, B.eps4[q], B.sig2[q]);
    }
    return lj_from_r2(r2, B.rc2, B.eps4[0], B.sig2[0]);
}

template <int W, int R, bool MIX>
__device__ __forceinline__ void eval_trial(const DevBox& B, const uint32_t* tab, int lg, const Trial& T,
                                           double& ea, double& eb, double* red, Work& wk) {
    const int tid = threadIdx.x;
    const int NS = B.nstencil << lg;
    const int two = (T.npos == 2 && !T.same) ? 1 : 0;
    const int total = NS << two;
    const int gmask = (1 << lg) - 1;
    const int32_t excl = (int32_t)T.idx;
    double sa = 0.0, sb = 0.0;
    for (int base = 0; base < total; base += kWave * W * R) {
        double4 e[R];
        int32_t cnt[R], kk[R], which[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int s = base + r * kWave * W + tid;
            const bool in = s < total;
            const int w = (two && s >= NS) ? 1 : 0;
            const int q = in ? s - w * NS : 0;
            const int t = q >> lg;
            const int k = q & gmask;
            const int32_t cx = w ? T.c[1][0] : T.c[0][0];
            const int32_t cy = w ? T.c[1][1] : T.c[0][1];
            const int32_t cz = w ? T.c[1][2] : T.c[0][2];
            const int64_t c = stencil_cell(B, tab[t], cx, cy, cz);
            const int kc = k < B.cap ? k : B.cap - 1;
            cnt[r] = in ? B.count[c] : 0;
            e[r] = B.ent[c * B.cap + kc];
            kk[r] = k;
            which[r] = w;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool valid = kk[r] < cnt[r] && meta_low(e[r].w) != excl;
            if (valid) {
                wk.cand += 1;
                if (T.npos == 1) {
                    sa += pair_energy_w<MIX>(B, T.p[0], T.sp, e[r], wk.incut);
                    wk.evals += 1;
                } else if (!two) {
                    sa += pair_energy_w<MIX>(B, T.p[0], T.sp, e[r], wk.incut);
                    sb += pair_energy_w<MIX>(B, T.p[1], T.sp, e[r], wk.incut);
                    wk.evals += 2;
                } else if (which[r]) {
                    sb += pair_energy_w<MIX>(B, T.p[1], T.sp, e[r], wk.incut);
                    wk.evals += 1;
                } else {
                    sa += pair_energy_w<MIX>(B, T.p[0], T.sp, e[r], wk.incut);
                    wk.evals += 1;
                }
            }
        }
    }
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    if (W == 1) {
        ea = sa;
        eb = sb;
        return;
    }
    const int wv = tid / kWave;
    if ((tid & (kWave - 1)) == 0) {
        red[2 * wv] = sa;
        red[2 * wv + 1] = sb;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int v = 0; v < W; ++v) {
        ta += red[2 * v];
        tb += red[2 * v + 1];
    }
    ea = ta;
    eb = tb;
}

// Remove the entry at `loc` of cell `c`: the cell's last entry takes its place
// (Sec. 3.2.5) and that particle's back-pointer follows.
__device__ __forceinline__ void remove_entry(const DevBox& B, int64_t c, int64_t loc) {
    const int32_t nc = B.count[c];
    const int64_t last = c * B.cap + nc - 1;
    if (loc != last) {
        const double4 e = B.ent[last];
        B.ent[loc] = e;
        B.pos[meta_low(e.w)].w = pack_meta(meta_species(e.w), (int32_t)loc);
    }
    B.count[c] = nc - 1;
}

// Apply an accepted trial (one thread).  Returns GCMC_OK, or an error with
// nothing written.  maxc is raised when a cell grows.
__device__ int commit_trial(const DevBox& B, const Trial& T, int64_t n, int32_t& maxc) {
    const int cap = B.cap;
    if (T.type == GCMC_MOVE_DISPLACE) {
        const int64_t loc = meta_low(T.meta);
        const double4 np = make_double4(T.p[1][0], T.p[1][1], T.p[1][2], 0.0);
        if (T.same) {
            B.ent[loc] = make_double4(np.x, np.y, np.z, pack_meta(T.sp, (int32_t)T.idx));
            B.pos[T.idx] = make_double4(np.x, np.y, np.z, T.meta);
            return GCMC_OK;
        }
        const int32_t nc = B.count[T.cl[1]];
        if (nc >= cap) return GCMC_ERR_CELL_OVERFLOW;
        remove_entry(B, T.cl[0], loc);
        const int64_t nl = T.cl[1] * cap + nc;
        B.ent[nl] = make_double4(np.x, np.y, np.z, pack_meta(T.sp, (int32_t)T.idx));
        B.count[T.cl[1]] = nc + 1;
        B.pos[T.idx] = make_double4(np.x, np.y, np.z, pack_meta(T.sp, (int32_t)nl));
        if (nc + 1 > maxc) maxc = nc + 1;
        return GCMC_OK;
    }
    if (T.type == GCMC_MOVE_INSERT) {
        if (n >= B.max_n) return GCMC_ERR_CAPACITY;
        const int32_t nc = B.count[T.cl[0]];
        if (nc >= cap) return GCMC_ERR_CELL_OVERFLOW;
        const int64_t nl = T.cl[0] * cap + nc;
        B.ent[nl] = make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(T.sp, (int32_t)n));
        B.count[T.cl[0]] = nc + 1;
        B.pos[n] = make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(T.sp, (int32_t)nl));
        if (nc + 1 > maxc) maxc = nc + 1;
        return GCMC_OK;
    }
    // deletion: drop the entry, then particle n-1 takes index idx
    const int64_t loc = meta_low(T.meta);
    remove_entry(B, T.cl[0], loc);
    if (T.idx != n - 1) {
        const double4 last = B.pos[n - 1];
        B.pos[T.idx] = last;
        const int64_t l2 = meta_low(last.w);
        B.ent[l2].w = pack_meta(meta_species(last.w), (int32_t)T.idx);
    }
    return GCMC_OK;
}

// ------------------------------------------------------------------ chain
// One workgroup advances one box by n_moves moves of Algorithm 1.
// boxes[blockIdx.x] is the box; its stats/log slot is order[blockIdx.x]
// (the caller's index of the box) or blockIdx.x.
template <int W, int R>
__global__ __launch_bounds__(kWave* W) void k_chain(const DevBox* __restrict__ boxes,
                                                     const int32_t* __restrict__ order, int64_t n_moves,
                                                     uint64_t ctr0, gcmc_stats* stats, gcmc_log* log) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ double red[2][2 * W];
    __shared__ int32_t sh_commit[2];
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;
    const DevBox& B = boxes[blockIdx.x];
    const int tid = threadIdx.x;
    BoxState* st = B.st;

    int64_t N = st->n;
    double U = st->u_pair;
    int32_t maxc = st->maxcount;
    int32_t err = st->error;
    int64_t err_move = st->error_move;
    int64_t att[3] = {0, 0, 0}, acc_n[3] = {0, 0, 0};
    double sum_n = 0.0, sum_u = 0.0;
    const double tk = B.tailK[0];
    int64_t m = 0;
    int ev = 0;   // evaluations done: selects the LDS reduction buffer
    int64_t stencils = 0;
    Work wk;
    build_stencil(B, tab);
    __syncthreads();
    if (err == GCMC_OK && B.ns == 1) {
        for (; m < n_moves; ++m) {
            const uint64_t ctr = ctr0 + (uint64_t)m;
            const U8 u = move_uniforms(B.seed, ctr, B.box_id);
            Trial T;
            T.type = (u.u[0] < B.p_disp) ? GCMC_MOVE_DISPLACE
                                         : ((u.u[1] < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
            T.sp = 0;
            att[T.type] += 1;
            if (T.type != GCMC_MOVE_INSERT && N == 0) {
                if (log && tid == 0) {
                    gcmc_log r;
                    r.type = T.type; r.index = -1; r.accepted = 0; r.flags = 1;
                    r.dU_pair = 0.0; r.dU_tail = 0.0; r.x = r.y = r.z = 0.0; r.arg = 0.0;
                    log[(size_t)bi * n_moves + m] = r;
                }
                sum_n += (double)N;
                sum_u += U + tk * (double)N * (double)N;
                continue;
            }
            if (T.type == GCMC_MOVE_INSERT) {
                T.idx = -1;
                T.npos = 1;
                T.same = 0;
                T.meta = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) T.p[0][a] = wrap_into_box(B.L[a] * u.u[4 + a], B.L[a]);
                locate(B, T, 0);
            } else {
                int64_t i = (int64_t)floor(u.u[2] * (double)N);
                if (i > N - 1) i = N - 1;
                T.idx = i;
                const double4 pi = B.pos[i];
                T.meta = pi.w;
                T.p[0][0] = pi.x; T.p[0][1] = pi.y; T.p[0][2] = pi.z;
                locate(B, T, 0);
                if (T.type == GCMC_MOVE_DISPLACE) {
                    T.npos = 2;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        T.p[1][a] = wrap_into_box(T.p[0][a] + B.max_disp * (2.0 * u.u[4 + a] - 1.0), B.L[a]);
                    locate(B, T, 1);
                    T.same = T.cl[0] == T.cl[1];
                } else {
                    T.npos = 1;
                    T.same = 0;
                }
            }
            double ea, eb;
            eval_trial<W, R, false>(B, tab, log2_ceil(maxc), T, ea, eb, red[ev & 1], wk);
            ++ev;
            stencils += (T.npos == 2 && !T.same) ? 2 : 1;
            double dUp, dUt;
            if (T.type == GCMC_MOVE_DISPLACE) {
                dUp = eb - ea;
                dUt = 0.0;
            } else if (T.type == GCMC_MOVE_INSERT) {
                dUp = ea;
                dUt = tk * (2.0 * (double)N + 1.0);
            } else {
                dUp = -ea;
                dUt = tk * (1.0 - 2.0 * (double)N);
            }
            const double dU = dUp + dUt;
            const double arg = accept_log_ratio(B, T.type, dU, N);
            const bool ok = metropolis(arg, dU, u.u[3]);
            if (ok) {
                if (tid == 0) {
                    int32_t mc = maxc;
                    sh_commit[0] = commit_trial(B, T, N, mc);
                    sh_commit[1] = mc;
                }
                __syncthreads();
                const int32_t e = sh_commit[0];
                maxc = sh_commit[1];
                __syncthreads();
                if (e != GCMC_OK) {
                    err = e;
                    err_move = (int64_t)ctr;
                    att[T.type] -= 1;
                    break;
                }
                acc_n[T.type] += 1;
                N += (T.type == GCMC_MOVE_INSERT) ? 1 : ((T.type == GCMC_MOVE_DELETE) ? -1 : 0);
                U += dUp;
            }
            if (log && tid == 0) {
                gcmc_log r;
                r.type = T.type;
                r.index = (T.type == GCMC_MOVE_INSERT) ? (int32_t)(N - (ok ? 1 : 0)) : (int32_t)T.idx;
                r.accepted = ok ? 1 : 0;
                r.flags = 0;
                r.dU_pair = dUp;
                r.dU_tail = dUt;
                const int w = (T.type == GCMC_MOVE_DISPLACE) ? 1 : 0;
                r.x = T.p[w][0]; r.y = T.p[w][1]; r.z = T.p[w][2];
                r.arg = arg;
                log[(size_t)bi * n_moves + m] = r;
            }
            sum_n += (double)N;
            sum_u += U + tk * (double)N * (double)N;
        }
    } else if (err == GCMC_OK) {
        err = GCMC_ERR_UNSUPPORTED;
        err_move = (int64_t)ctr0;
    }
    // launch-wide work counters: wavefront sums, then LDS across wavefronts
    __shared__ int64_t wred[3][W];
    {
        int64_t c = wk.cand, e = wk.evals, q = wk.incut;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            c += __shfl_xor(c, off, kWave);
            e += __shfl_xor(e, off, kWave);
            q += __shfl_xor(q, off, kWave);
        }
        __syncthreads();
        if ((tid & (kWave - 1)) == 0) {
            wred[0][tid / kWave] = c;
            wred[1][tid / kWave] = e;
            wred[2][tid / kWave] = q;
        }
        __syncthreads();
    }
    if (tid == 0) {
        st->n = N;
        st->u_pair = U;
        st->maxcount = maxc;
        st->nsp[0] = N;
        if (err != GCMC_OK && st->error == GCMC_OK) {
            st->error = err;
            st->error_move = err_move;
        }
        if (stats) {
            gcmc_stats o;
            for (int t = 0; t < 3; ++t) {
                o.attempts[t] = att[t];
                o.accepts[t] = acc_n[t];
            }
            o.n = N;
            o.moves_done = m;
            o.u_pair = U;
            o.u_tail = tk * (double)N * (double)N;
            o.sum_n = sum_n;
            o.sum_u = sum_u;
            o.error = st->error;
            o.pad = 0;
            o.error_move = st->error_move;
            o.stencils = stencils;
            o.candidates = o.pair_evals = o.in_cutoff = 0;
            for (int v = 0; v < W; ++v) {
                o.candidates += wred[0][v];
                o.pair_evals += wred[1][v];
                o.in_cutoff += wred[2][v];
            }
            stats[bi] = o;
        }
    }
}

// ---------------------------------------------------- host-driven moves
// Build the trial of a caller-given move against the current state.  Returns
// false (trial unusable) for an out-of-range index or species.
__device__ __forceinline__ bool trial_from_move(const DevBox& B, const gcmc_move& mv, int64_t n, Trial& T) {
    T.type = mv.type;
    if (mv.type == GCMC_MOVE_INSERT) {
        if (mv.species < 0 || mv.species >= B.ns) return false;
        T.sp = mv.species;
        T.idx = -1;
        T.npos = 1;
        T.same = 0;
        T.meta = 0.0;
        T.p[0][0] = mv.x; T.p[0][1] = mv.y; T.p[0][2] = mv.z;
        locate(B, T, 0);
        return true;
    }
    if (mv.type != GCMC_MOVE_DISPLACE && mv.type != GCMC_MOVE_DELETE) return false;
    if (mv.index < 0 || mv.index >= n) return false;
    T.idx = mv.index;
    const double4 pi = B.pos[T.idx];
    T.meta = pi.w;
    T.sp = meta_species(pi.w);
    T.p[0][0] = pi.x; T.p[0][1] = pi.y; T.p[0][2] = pi.z;
    locate(B, T, 0);
    if (mv.type == GCMC_MOVE_DISPLACE) {
        T.npos = 2;
        T.p[1][0] = mv.x; T.p[1][1] = mv.y; T.p[1][2] = mv.z;
        locate(B, T, 1);
        T.same = T.cl[0] == T.cl[1];
    } else {
        T.npos = 1;
        T.same = 0;
    }
    return true;
}

template <int W, int R, bool MIX>
__global__ __launch_bounds__(kWave* W) void k_delta(const DevBox* __restrict__ boxp, const gcmc_move* moves,
                                                     int64_t n_moves, double* dU_pair, double* dU_tail) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ double red[2 * W];
    const DevBox& B = *boxp;
    build_stencil(B, tab);
    __syncthreads();
    const int64_t n = B.st->n;
    int64_t nsp[kMaxSpecies];
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) nsp[s] = B.st->nsp[s];
    const int lg = log2_ceil(B.st->maxcount);
    for (int64_t m = blockIdx.x; m < n_moves; m += gridDim.x) {
        const gcmc_move mv = moves[m];
        Trial T;
        const bool ok = trial_from_move(B, mv, n, T);
        double ea = 0.0, eb = 0.0;
        Work wk;
        if (ok) eval_trial<W, R, MIX>(B, tab, lg, T, ea, eb, red, wk);
        __syncthreads();
        if (threadIdx.x == 0) {
            double p, t;
            if (!ok) {
                p = __builtin_nan("");
                t = __builtin_nan("");
            } else if (T.type == GCMC_MOVE_DISPLACE) {
                p = eb - ea;
                t = 0.0;
            } else if (T.type == GCMC_MOVE_INSERT) {
                p = ea;
                t = tail_change(B, nsp, T.sp, +1);
            } else {
                p = -ea;
                t = tail_change(B, nsp, T.sp, -1);
            }
            dU_pair[m] = p;
            if (dU_tail) dU_tail[m] = t;
        }
    }
}

__global__ void k_commit(const DevBox* __restrict__ boxp, const gcmc_move* move, const double* dU_pair) {
    const DevBox& B = *boxp;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    BoxState* st = B.st;
    if (st->error != GCMC_OK) return;
    const int64_t n = st->n;
    const gcmc_move mv = *move;
    Trial T;
    if (!trial_from_move(B, mv, n, T)) {
        st->error = GCMC_ERR_INVALID_ARG;
        st->error_move = -1;
        return;
    }
    int32_t mc = st->maxcount;
    const int e = commit_trial(B, T, n, mc);
    if (e != GCMC_OK) {
        st->error = e;
        st->error_move = -1;
        return;
    }
    st->maxcount = mc;
    if (T.type == GCMC_MOVE_INSERT) {
        st->n = n + 1;
        st->nsp[T.sp] += 1;
    } else if (T.type == GCMC_MOVE_DELETE) {
        st->n = n - 1;
        st->nsp[T.sp] -= 1;
    }
    st->u_pair += *dU_pair;
}

// Candidate ids of points (the same slot mapping as eval_trial).
__global__ __launch_bounds__(256) void k_neighbors(const DevBox* __restrict__ boxp, const double* pts,
                                                   const int32_t* excl, int64_t n, int32_t max_ids, int32_t* ids,
                                                   int32_t* counts) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ int32_t fill;
    const DevBox& B = *boxp;
    build_stencil(B, tab);
    const int lg = log2_ceil(B.st->maxcount);
    const int NS = B.nstencil << lg;
    const int gmask = (1 << lg) - 1;
    for (int64_t m = blockIdx.x; m < n; m += gridDim.x) {
        if (threadIdx.x == 0) fill = 0;
        __syncthreads();
        Trial T;
        T.p[0][0] = pts[m]; T.p[0][1] = pts[n + m]; T.p[0][2] = pts[2 * n + m];
        locate(B, T, 0);
        const int32_t ex = excl ? excl[m] : -1;
        for (int s = threadIdx.x; s < NS; s += blockDim.x) {
            const int t = s >> lg, k = s & gmask;
            const int64_t c = stencil_cell(B, tab[t], T.c[0][0], T.c[0][1], T.c[0][2]);
            if (k < B.count[c] && k < B.cap) {
                const int32_t id = meta_low(B.ent[c * B.cap + k].w);
                if (id != ex) {
                    const int32_t at = atomicAdd(&fill, 1);
                    if (at < max_ids) ids[m * max_ids + at] = id;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) counts[m] = fill;
        __syncthreads();
    }
}

// ---------------------------------------------------------- dispatch
using chain_fn = void (*)(const DevBox*, const int32_t*, int64_t, uint64_t, gcmc_stats*, gcmc_log*);
using delta_fn = void (*)(const DevBox*, const gcmc_move*, int64_t, double*, double*);

struct ChainCfg {
    int w, r;
    chain_fn f;
};

static const ChainCfg kChainCfgs[] = {
    {1, 8, k_chain<1, 8>},  {2, 8, k_chain<2, 8>},  {4, 2, k_chain<4, 2>},
    {4, 4, k_chain<4, 4>}, {4, 8, k_chain<4, 8>},   {8, 2, k_chain<8, 2>},  {8, 4, k_chain<8, 4>},
    {16, 2, k_chain<16, 2>},
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

int launch_delta(const DevBox* d_box, bool mix, int64_t n_moves, const gcmc_move* moves, double* dp, double* dt,
                 hipStream_t s) {
    const int64_t g64 = n_moves < 65536 ? n_moves : 65536;
    const int g = (int)(g64 < 1 ? 1 : g64);
    if (mix)
        hipLaunchKernelGGL((k_delta<4, 4, true>), dim3(g), dim3(kWave * 4), 0, s, d_box, moves, n_moves, dp, dt);
    else
        hipLaunchKernelGGL((k_delta<4, 4, false>), dim3(g), dim3(kWave * 4), 0, s, d_box, moves, n_moves, dp, dt);
    return 0;
}

void launch_commit(const DevBox* d_box, const gcmc_move* move, const double* dU, hipStream_t s) {
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, s, d_box, move, dU);
}

void launch_neighbors(const DevBox* d_box, const double* pts, const int32_t* excl, int64_t n, int32_t max_ids,
                      int32_t* ids, int32_t* counts, hipStream_t s) {
    const int64_t g64 = n < 65536 ? n : 65536;
    hipLaunchKernelGGL(k_neighbors, dim3((int)(g64 < 1 ? 1 : g64)), dim3(256), 0, s, d_box, pts, excl, n, max_ids,
                       ids, counts);
}

}  // namespace gcmc
