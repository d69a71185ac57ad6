// The persistent chain of Algorithm 1 for a small box held in local memory.
//
// In a box of a few hundred to a couple of thousand particles the 27-cell
// stencil covers most or all of the box, so the cell list prunes little, and a
// move of the global-memory kernels is a chain of dependent memory round trips
// (pick record, counters, candidates, commit) of roughly a microsecond each.
// Here one workgroup copies the box's coordinates into LDS once per launch and
// runs every move against that copy: all W wavefronts evaluate one move
// together (each takes every (64 W)-th particle, the in-cutoff pairs queued
// and evaluated 64 at a time), the per-wavefront sums are added in a fixed
// order, every thread takes the same Metropolis decision, and an accepted
// move is committed to the LDS copy by one thread.  The energy of a move is
// the sum over all other particles inside the cutoff (Eq. 1 with the strict
// cutoff), the same set of pairs the cell list finds.  Particles with an index
// of kResCap or more (a box that grows past it) are read from and written to
// global memory instead: correct, only slower.
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

template <int W>
__global__ __launch_bounds__(kWave* W) void k_chain_resident(const DevBox* __restrict__ boxes,
                                                              const int32_t* __restrict__ order, int64_t n_moves,
                                                              uint64_t ctr0, gcmc_stats* stats, gcmc_log* trace) {
    __shared__ double px[kResCap], py[kResCap], pz[kResCap];
    __shared__ DrawRing<kResRing> dring;
    __shared__ ResMove mv[kResRing];
    // log acceptance prefactors for N = lbase + t: insertion V / (Lambda^3 (N + 1)), deletion
    // Lambda^3 N / V (N moves by at most one per move, so kResRing moves stay inside)
    __shared__ double lpi[2 * kResRing + 1], lpd[2 * kResRing + 1];
    __shared__ double red[2][W][4];       // per-wavefront sums of the move, two buffers
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
    int64_t att0 = 0, att1 = 0, att2 = 0, acc0 = 0, acc1 = 0, acc2 = 0;
    double sum_n = 0.0, sum_u = 0.0, sum_n2 = 0.0, sum_w = 0.0;
    int64_t cand = 0, evals = 0, incut = 0;

    auto get = [&](int64_t j) -> double3 {
        if (j < kResCap) return make_double3(px[j], py[j], pz[j]);
        return gload_xyz(B.pos + j);
    };
    auto put = [&](int64_t j, double x, double y, double z) {
        if (j < kResCap) {
            px[j] = x;
            py[j] = y;
            pz[j] = z;
        } else {
            gstore(B.pos + j, make_double4(x, y, z, 0.0));
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
    if (err == GCMC_OK && B.ns != 1) {
        err = GCMC_ERR_UNSUPPORTED;
        err_move = (int64_t)ctr0;
    }
    int64_t m = 0;
    int64_t lbase = 0;
    while (err == GCMC_OK && m < n_moves) {
        const uint64_t ctr = ctr0 + (uint64_t)m;
        if ((m & (kResRing - 1)) == 0) {
            // moves m .. m + kResRing - 1: Philox block t & 3 of move m + t / 4 per thread, then one
            // thread per move derives what the move needs; the prefactor tables for every N these
            // moves can meet (every thread has read the previous entries: the barrier before)
            __syncthreads();
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
            __syncthreads();
        }
        const int s = (int)(ctr & (uint64_t)(kResRing - 1));
        const int type = uni(mv[s].type);
        if (type == GCMC_MOVE_DISPLACE) att0 += 1;
        else if (type == GCMC_MOVE_INSERT) att1 += 1;
        else att2 += 1;
        // ------------------------------------------------ empty box: rejection
        if (type != GCMC_MOVE_INSERT && N == 0) {
            if (trace && tid == 0) {
                gcmc_log r;
                r.type = type; r.index = -1; r.accepted = 0; r.flags = 1;
                r.dU_pair = 0.0; r.dU_tail = 0.0; r.x = r.y = r.z = 0.0; r.arg = 0.0; r.dW_pair = 0.0;
                trace[(size_t)bi * n_moves + m] = r;
            }
            sum_u += U;
            sum_w += Wvir;
            ++m;
            continue;
        }
        // ------------------------------------------------ the trial position(s)
        int64_t idx = -1;
        double p0[3], p1[3] = {0.0, 0.0, 0.0};
        if (type == GCMC_MOVE_INSERT) {
#pragma unroll
            for (int a = 0; a < 3; ++a) p0[a] = mv[s].q[a];
        } else {
            // the pick (reading 9 of the design notes' pick rule) on scalar integers; the floor of
            // u2 N only when no field is below N
            const uint64_t k = ((uint64_t)uni((int32_t)mv[s].khi) << 32) | (uint32_t)uni((int32_t)mv[s].klo);
            if (N == 1) {
                idx = 0;
            } else {
                const int b = 64 - __clzll((long long)(N - 1));
                const uint64_t mask = (1ull << b) - 1ull;
                for (int sh = 53 - b; sh >= 0 && idx < 0; sh -= b) {
                    const uint64_t v = (k >> sh) & mask;
                    if (v < (uint64_t)N) idx = (int64_t)v;
                }
                if (idx < 0) {
                    const int64_t i = (int64_t)floor(mv[s].u2 * (double)N);
                    idx = uni64(i > N - 1 ? N - 1 : i);
                }
            }
            const double3 o = get(idx);
            p0[0] = o.x; p0[1] = o.y; p0[2] = o.z;
            if (type == GCMC_MOVE_DISPLACE) {
#pragma unroll
                for (int a = 0; a < 3; ++a) p1[a] = wrap_into_box(p0[a] + mv[s].q[a], B.L[a]);
            }
        }
        // ------------------------------------------------ pair sums over every other particle
        const bool disp = type == GCMC_MOVE_DISPLACE;
        double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
        int32_t n_in = 0, n_eval = 0;
        for (int64_t j0 = (int64_t)wv * kWave; j0 < N; j0 += (int64_t)blockDim.x) {
            const int64_t j = j0 + lane;
            const bool valid = j < N && j != idx;
            const double3 e = valid ? get(j) : make_double3(p0[0] + B.L[0] * 0.5, p0[1], p0[2]);
            cand += valid ? 1 : 0;
            n_eval += valid ? (disp ? 2 : 1) : 0;
            const double r2a = spec_dist2(B, p0, e, true);
            pair(valid ? r2a : rc2, sa, wa, n_in);
            if (disp) {
                const double r2b = spec_dist2(B, p1, e, true);
                pair(valid ? r2b : rc2, sb, wb, n_in);
            }
        }
        evals += n_eval;
        incut += n_in;
        const int rb = (int)(m & 1);
        sa = wave_sum_uniform(sa);
        sb = wave_sum_uniform(sb);
        wa = wave_sum_uniform(wa);
        wb = wave_sum_uniform(wb);
        if (lane == 0) {
            red[rb][wv][0] = sa;
            red[rb][wv][1] = sb;
            red[rb][wv][2] = wa;
            red[rb][wv][3] = wb;
        }
        __syncthreads();
        double ea = 0.0, eb = 0.0, va = 0.0, vb = 0.0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            ea += red[rb][v][0];
            eb += red[rb][v][1];
            va += red[rb][v][2];
            vb += red[rb][v][3];
        }
        // ------------------------------------------------ decide (Eqs. 3-5), the same in every thread
        const bool is_ins = type == GCMC_MOVE_INSERT;
        const double dUp = disp ? (eb - ea) : (is_ins ? ea : -ea);
        const double dWp = disp ? (vb - va) : (is_ins ? va : -va);
        const double dUt = disp ? 0.0 : tk * (is_ins ? (2.0 * (double)N + 1.0) : (1.0 - 2.0 * (double)N));
        const double dU = dUp + dUt;
        const double lpref = disp ? 0.0 : (is_ins ? lpi[N - lbase] : lpd[N - lbase]);
        const double arg = disp ? -(B.beta * dU) : (is_ins ? lpref + B.beta * (B.mu - dU) : lpref - B.beta * (B.mu + dU));
        const bool ok = __builtin_amdgcn_readfirstlane((dU == dU && mv[s].lnA < arg) ? 1 : 0) != 0;
        const int64_t n_old = N;
        if (ok) {
            if (is_ins && N >= B.max_n) {
                err = GCMC_ERR_CAPACITY;
                err_move = (int64_t)ctr;
                att1 -= 1;
                break;
            }
            if (tid == 0) {
                if (is_ins) {
                    put(N, p0[0], p0[1], p0[2]);
                } else if (disp) {
                    put(idx, p1[0], p1[1], p1[2]);
                } else if (idx != N - 1) {
                    // particle N-1 takes index idx
                    const double3 l = get(N - 1);
                    put(idx, l.x, l.y, l.z);
                }
            }
            if (disp) acc0 += 1;
            else if (is_ins) acc1 += 1;
            else acc2 += 1;
            N += is_ins ? 1 : (disp ? 0 : -1);
            U += dUp;
            Wvir += dWp;
            __syncthreads();   // the commit visible to every wavefront
        }
        if (trace && tid == 0) {
            gcmc_log r;
            r.type = type;
            r.index = is_ins ? (int32_t)n_old : (int32_t)idx;
            r.accepted = ok ? 1 : 0;
            r.flags = 0;
            r.dU_pair = dUp;
            r.dU_tail = dUt;
            const double* q = disp ? p1 : p0;
            r.x = q[0]; r.y = q[1]; r.z = q[2];
            r.arg = arg;
            r.dW_pair = dWp;
            trace[(size_t)bi * n_moves + m] = r;
        }
        sum_n += (double)N;
        sum_n2 += (double)N * (double)N;
        sum_u += U + tk * (double)N * (double)N;
        sum_w += Wvir;
        ++m;
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
