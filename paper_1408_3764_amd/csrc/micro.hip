// The paper's microcell thread mapping (Sec. 3.3, 3.3.2): one move at a time,
// each thread of the workgroup takes one cell of the move's stencil -- the
// cube of cells around the particle's cell, here without the cells beyond the
// cutoff -- and loops over the particles in it; when the stencil has more
// cells than the workgroup has threads, the threads iterate over several
// cells.  The energies are reduced over the workgroup (wavefront sums, then
// the wavefronts' sums in a fixed order); the draws, the acceptance and the
// incremental cell update are those of the other chain kernels.  Kept beside
// the candidate-per-lane kernels to compare the two mappings on the same
// grids.
#include "trial.h"

namespace gcmc {

template <int W>
__global__ __launch_bounds__(kWave* W) void k_chain_paper(const DevBox* __restrict__ boxes,
                                                           const int32_t* __restrict__ order, int64_t n_moves,
                                                           uint64_t ctr0, gcmc_stats* stats, gcmc_log* trace) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ double red[4 * W];
    __shared__ int32_t sh_err;
    __shared__ int32_t sh_maxc;
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;
    const DevBox B = hot_copy(boxes[blockIdx.x]);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
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
    int64_t att[3] = {0, 0, 0}, acc[3] = {0, 0, 0};
    double sum_n = 0.0, sum_u = 0.0, sum_n2 = 0.0, sum_w = 0.0;
    int64_t stencils = 0, cand = 0, evals = 0, incut = 0;   // per thread, added up at the end
    load_stencil(B, tab);
    __syncthreads();
    if (err == GCMC_OK && B.ns != 1) {
        err = GCMC_ERR_UNSUPPORTED;
        err_move = (int64_t)ctr0;
    }
    int64_t m = 0;
    for (; err == GCMC_OK && m < n_moves; ++m) {
        const uint64_t ctr = ctr0 + (uint64_t)m;
        const U8 u = move_uniforms(B.seed, ctr, B.box_id);
        const int type = (u.u[0] < B.p_disp) ? GCMC_MOVE_DISPLACE : ((u.u[1] < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
        att[type] += 1;
        if (type != GCMC_MOVE_INSERT && N == 0) {
            if (trace && tid == 0) {
                gcmc_log r;
                r.type = type; r.index = -1; r.accepted = 0; r.flags = 1;
                r.dU_pair = 0.0; r.dU_tail = 0.0; r.x = r.y = r.z = 0.0; r.arg = 0.0; r.dW_pair = 0.0;
                trace[(size_t)bi * n_moves + m] = r;
            }
            sum_u += U;
            sum_w += Wvir;
            continue;
        }
        // the trial
        Trial T;
        T.type = type;
        T.sp = 0;
        if (type == GCMC_MOVE_INSERT) {
            T.idx = -1;
            T.npos = 1;
            T.same = 0;
            T.meta = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) T.p[0][a] = wrap_into_box(B.L[a] * u.u[4 + a], B.L[a]);
            locate(B, T, 0);
        } else {
            T.idx = pick_particle(u.u[2], u.u[7], N);
            const double4 rec = gload(B.pos + T.idx);
            T.meta = rec.w;
            T.p[0][0] = rec.x; T.p[0][1] = rec.y; T.p[0][2] = rec.z;
            locate(B, T, 0);
            if (type == GCMC_MOVE_DISPLACE) {
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
        const int two = (T.npos == 2 && !T.same) ? 1 : 0;
        const int ncell = B.nstencil << two;
        const int32_t excl = (int32_t)T.idx;
        // one thread per stencil cell, a loop over the particles in it
        double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
        for (int f = tid; f < ncell; f += blockDim.x) {
            const int w = f >= B.nstencil ? 1 : 0;
            const int t = f - w * B.nstencil;
            const int64_t c = stencil_cell(B, tab[t], T.c[w][0], T.c[w][1], T.c[w][2]);
            int32_t cnt = gload(B.count + c);
            cnt = cnt < cap ? cnt : cap;
            for (int32_t k = 0; k < cnt; ++k) {
                const double4 e = gload(B.ent + (c * cap + k));
                if (meta_low(e.w) == excl) continue;
                cand += 1;
                if (T.npos == 1) {
                    sa += pair_uw<false>(B, T.p[0], 0, e, incut, wa);
                    evals += 1;
                } else if (!two) {
                    sa += pair_uw<false>(B, T.p[0], 0, e, incut, wa);
                    sb += pair_uw<false>(B, T.p[1], 0, e, incut, wb);
                    evals += 2;
                } else if (w) {
                    sb += pair_uw<false>(B, T.p[1], 0, e, incut, wb);
                    evals += 1;
                } else {
                    sa += pair_uw<false>(B, T.p[0], 0, e, incut, wa);
                    evals += 1;
                }
            }
        }
        if (tid == 0) stencils += two ? 2 : 1;
        sa = wave_sum(sa);
        sb = wave_sum(sb);
        wa = wave_sum(wa);
        wb = wave_sum(wb);
        if (lane == 0) {
            red[4 * wv] = sa;
            red[4 * wv + 1] = sb;
            red[4 * wv + 2] = wa;
            red[4 * wv + 3] = wb;
        }
        __syncthreads();
        double ea = 0.0, eb = 0.0, va = 0.0, vb = 0.0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            ea += red[4 * v];
            eb += red[4 * v + 1];
            va += red[4 * v + 2];
            vb += red[4 * v + 3];
        }
        // the decision (Eqs. 3-5), the same in every thread
        const bool is_disp = type == GCMC_MOVE_DISPLACE, is_ins = type == GCMC_MOVE_INSERT;
        const double dUp = is_disp ? (eb - ea) : (is_ins ? ea : -ea);
        const double dWp = is_disp ? (vb - va) : (is_ins ? va : -va);
        const double dUt = is_disp ? 0.0 : tk * (is_ins ? (2.0 * (double)N + 1.0) : (1.0 - 2.0 * (double)N));
        const double dU = dUp + dUt;
        const double arg = accept_log_ratio(B, type, dU, N);
        const bool ok = metropolis(arg, dU, u.u[3]);
        const int64_t n_old = N;
        if (ok) {
            if (tid == 0) {
                int32_t mc = maxc;
                sh_err = commit_trial(B, T, N, mc);
                sh_maxc = mc;
            }
            __syncthreads();   // the commit's stores done and visible to the workgroup
            const int e = sh_err;
            if (e != GCMC_OK) {
                err = e;
                err_move = (int64_t)ctr;
                att[type] -= 1;
                break;
            }
            maxc = sh_maxc;
            acc[type] += 1;
            N += is_ins ? 1 : (type == GCMC_MOVE_DELETE ? -1 : 0);
            U += dUp;
            Wvir += dWp;
        } else {
            __syncthreads();   // red[] read by every thread before the next move writes it
        }
        if (trace && tid == 0) {
            gcmc_log r;
            r.type = type;
            r.index = is_ins ? (int32_t)n_old : (int32_t)T.idx;
            r.accepted = ok ? 1 : 0;
            r.flags = 0;
            r.dU_pair = dUp;
            r.dU_tail = dUt;
            const int w = is_disp ? 1 : 0;
            r.x = T.p[w][0]; r.y = T.p[w][1]; r.z = T.p[w][2];
            r.arg = arg;
            r.dW_pair = dWp;
            trace[(size_t)bi * n_moves + m] = r;
        }
        sum_n += (double)N;
        sum_n2 += (double)N * (double)N;
        sum_u += U + tk * (double)N * (double)N;
        sum_w += Wvir;
    }
    // work counters over the workgroup (fixed order)
    __shared__ int64_t wred[4][W];
    {
        int64_t c = cand, e = evals, q = incut, sx = stencils;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            c += __shfl_xor(c, off, kWave);
            e += __shfl_xor(e, off, kWave);
            q += __shfl_xor(q, off, kWave);
            sx += __shfl_xor(sx, off, kWave);
        }
        __syncthreads();
        if (lane == 0) {
            wred[0][wv] = c;
            wred[1][wv] = e;
            wred[2][wv] = q;
            wred[3][wv] = sx;
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
            L.acc[t] = acc[t];
        }
        L.sum_n = sum_n;
        L.sum_n2 = sum_n2;
        L.sum_u = sum_u;
        L.sum_w = sum_w;
        int64_t c = 0, e = 0, q = 0, sx = 0;
        for (int v = 0; v < W; ++v) {
            c += wred[0][v];
            e += wred[1][v];
            q += wred[2][v];
            sx += wred[3][v];
        }
        finish_launch(B, st, L, N, U, Wvir, sx, c, e, q, stats ? stats + bi : nullptr);
    }
}

using paper_fn = void (*)(const DevBox*, const int32_t*, int64_t, uint64_t, gcmc_stats*, gcmc_log*);

struct PaperCfg {
    int w;
    paper_fn f;
};

static const PaperCfg kPaperCfgs[] = {{4, k_chain_paper<4>}, {8, k_chain_paper<8>}};

bool paper_cfg_exists(int waves) {
    for (const PaperCfg& c : kPaperCfgs)
        if (c.w == waves) return true;
    return false;
}

int launch_chain_paper(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                       uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s) {
    for (const PaperCfg& c : kPaperCfgs) {
        if (c.w == waves) {
            hipLaunchKernelGGL(c.f, dim3(n_boxes), dim3(kWave * c.w), 0, s, d_boxes, d_order, n_moves, ctr0, stats,
                               log);
            return 0;
        }
    }
    return -1;
}

}  // namespace gcmc
