// Host-driven move kernels: energy deltas of caller-given trial moves, the
// commit of one accepted move, and the neighbour-candidate gather (the same
// stencil mapping as the energy evaluation, for checking it).
#include "trial.h"

namespace gcmc {

template <int W, int R, bool MIX>
__global__ __launch_bounds__(kWave* W) void k_delta(const DevBox* __restrict__ boxp, const gcmc_move* moves,
                                                     int64_t n_moves, double* dU_pair, double* dU_tail,
                                                     double* dW_pair) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ double red[4 * W];
    const DevBox& B = *boxp;
    load_stencil(B, tab);
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
        double ea = 0.0, eb = 0.0, va = 0.0, vb = 0.0;
        Work wk;
        if (ok) eval_trial<W, R, MIX>(B, tab, lg, T, ea, eb, va, vb, red, wk);
        __syncthreads();
        if (threadIdx.x == 0) {
            double p, t, w;
            if (!ok) {
                p = __builtin_nan("");
                t = __builtin_nan("");
                w = __builtin_nan("");
            } else if (T.type == GCMC_MOVE_DISPLACE) {
                p = eb - ea;
                t = 0.0;
                w = vb - va;
            } else if (T.type == GCMC_MOVE_INSERT) {
                p = ea;
                t = tail_change(B, nsp, T.sp, +1);
                w = va;
            } else {
                p = -ea;
                t = tail_change(B, nsp, T.sp, -1);
                w = -va;
            }
            dU_pair[m] = p;
            if (dU_tail) dU_tail[m] = t;
            if (dW_pair) dW_pair[m] = w;
        }
    }
}

__global__ void k_commit(const DevBox* __restrict__ boxp, const gcmc_move* move, const double* dU_pair,
                         const double* dW_pair) {
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
    st->w_pair = dW_pair ? st->w_pair + *dW_pair : __builtin_nan("");
}

// Candidate ids of points (the same slot mapping as eval_trial).
__global__ __launch_bounds__(256) void k_neighbors(const DevBox* __restrict__ boxp, const double* pts,
                                                   const int32_t* excl, int64_t n, int32_t max_ids, int32_t* ids,
                                                   int32_t* counts) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ int32_t fill;
    const DevBox& B = *boxp;
    load_stencil(B, tab);
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
            if (k < gload(B.count + c) && k < B.cap) {
                const int32_t id = meta_low(gload(B.ent + (c * B.cap + k)).w);
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
int launch_delta(const DevBox* d_box, bool mix, int64_t n_moves, const gcmc_move* moves, double* dp, double* dt,
                 double* dw, hipStream_t s) {
    const int64_t g64 = n_moves < 65536 ? n_moves : 65536;
    const int g = (int)(g64 < 1 ? 1 : g64);
    if (mix)
        hipLaunchKernelGGL((k_delta<4, 4, true>), dim3(g), dim3(kWave * 4), 0, s, d_box, moves, n_moves, dp, dt, dw);
    else
        hipLaunchKernelGGL((k_delta<4, 4, false>), dim3(g), dim3(kWave * 4), 0, s, d_box, moves, n_moves, dp, dt, dw);
    return 0;
}

void launch_commit(const DevBox* d_box, const gcmc_move* move, const double* dU, const double* dW, hipStream_t s) {
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, s, d_box, move, dU, dW);
}

void launch_neighbors(const DevBox* d_box, const double* pts, const int32_t* excl, int64_t n, int32_t max_ids,
                      int32_t* ids, int32_t* counts, hipStream_t s) {
    const int64_t g64 = n < 65536 ? n : 65536;
    hipLaunchKernelGGL(k_neighbors, dim3((int)(g64 < 1 ? 1 : g64)), dim3(256), 0, s, d_box, pts, excl, n, max_ids,
                       ids, counts);
}

}  // namespace gcmc
