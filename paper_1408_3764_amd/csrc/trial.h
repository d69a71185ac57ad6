// Trial moves: their setup, the energy evaluation over the cell stencil, and
// the incremental cell update on acceptance (shared by the host-driven move
// kernels and the persistent chain kernel).
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
#pragma once

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

// Pair energy and pair virial together (the virial added to `w`).
template <bool MIX>
__device__ __forceinline__ double pair_uw(const DevBox& B, const double* p, int sp, const double4& e, int64_t& incut,
                                          double& w) {
    const double r2 = dist2(B, p[0], p[1], p[2], e.x, e.y, e.z);
    incut += (r2 < B.rc2) ? 1 : 0;
    if (MIX) {
        const int q = sp * B.ns + meta_species(e.w);
        return lj_uw_from_r2(r2, B.rc2, B.eps4[q], B.sig2[q], w);
    }
    return lj_uw_from_r2(r2, B.rc2, B.eps4[0], B.sig2[0], w);
}

// Block-wide: ea = sum over candidates of u(p[0], .), eb = sum of u(p[1], .)
// (eb only for displacements), va and vb the same sums of the pair virial.
// `red` holds 4*W doubles of LDS.
template <int W, int R, bool MIX>
__device__ __forceinline__ void eval_trial(const DevBox& B, const uint32_t* tab, int lg, const Trial& T,
                                           double& ea, double& eb, double& va, double& vb, double* red, Work& wk) {
    const int tid = threadIdx.x;
    const int NS = B.nstencil << lg;
    const int two = (T.npos == 2 && !T.same) ? 1 : 0;
    const int total = NS << two;
    const int gmask = (1 << lg) - 1;
    const int32_t excl = (int32_t)T.idx;
    double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
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
            cnt[r] = in ? gload(B.count + c) : 0;
            e[r] = gload(B.ent + (c * B.cap + kc));
            kk[r] = k;
            which[r] = w;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool valid = kk[r] < cnt[r] && meta_low(e[r].w) != excl;
            if (valid) {
                wk.cand += 1;
                if (T.npos == 1) {
                    sa += pair_uw<MIX>(B, T.p[0], T.sp, e[r], wk.incut, wa);
                    wk.evals += 1;
                } else if (!two) {
                    sa += pair_uw<MIX>(B, T.p[0], T.sp, e[r], wk.incut, wa);
                    sb += pair_uw<MIX>(B, T.p[1], T.sp, e[r], wk.incut, wb);
                    wk.evals += 2;
                } else if (which[r]) {
                    sb += pair_uw<MIX>(B, T.p[1], T.sp, e[r], wk.incut, wb);
                    wk.evals += 1;
                } else {
                    sa += pair_uw<MIX>(B, T.p[0], T.sp, e[r], wk.incut, wa);
                    wk.evals += 1;
                }
            }
        }
    }
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    wa = wave_sum(wa);
    wb = wave_sum(wb);
    if (W == 1) {
        ea = sa;
        eb = sb;
        va = wa;
        vb = wb;
        return;
    }
    const int wv = tid / kWave;
    if ((tid & (kWave - 1)) == 0) {
        red[4 * wv] = sa;
        red[4 * wv + 1] = sb;
        red[4 * wv + 2] = wa;
        red[4 * wv + 3] = wb;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0, ua = 0.0, ub = 0.0;
#pragma unroll
    for (int v = 0; v < W; ++v) {
        ta += red[4 * v];
        tb += red[4 * v + 1];
        ua += red[4 * v + 2];
        ub += red[4 * v + 3];
    }
    ea = ta;
    eb = tb;
    va = ua;
    vb = ub;
}

// Remove the entry at `loc` of cell `c`: the cell's last entry takes its place
// (Sec. 3.2.5) and that particle's back-pointer follows.
__device__ __forceinline__ void remove_entry(const DevBox& B, int64_t c, int64_t loc) {
    const int32_t nc = gload(B.count + c);
    const int64_t last = c * B.cap + nc - 1;
    if (loc != last) {
        const double4 e = gload(B.ent + last);
        gstore(B.ent + loc, e);
        gstore_w(B.pos + (meta_low(e.w)), pack_meta(meta_species(e.w), (int32_t)loc));
    }
    gstore(B.count + c, nc - 1);
}

// Apply an accepted trial (one thread).  Returns GCMC_OK, or an error with
// nothing written.  maxc is raised when a cell grows.
__device__ int commit_trial(const DevBox& B, const Trial& T, int64_t n, int32_t& maxc) {
    const int cap = B.cap;
    if (T.type == GCMC_MOVE_DISPLACE) {
        const int64_t loc = meta_low(T.meta);
        const double4 np = make_double4(T.p[1][0], T.p[1][1], T.p[1][2], 0.0);
        if (T.same) {
            gstore(B.ent + loc, make_double4(np.x, np.y, np.z, pack_meta(T.sp, (int32_t)T.idx)));
            gstore(B.pos + T.idx, make_double4(np.x, np.y, np.z, T.meta));
            return GCMC_OK;
        }
        const int32_t nc = gload(B.count + (T.cl[1]));
        if (nc >= cap) return GCMC_ERR_CELL_OVERFLOW;
        remove_entry(B, T.cl[0], loc);
        const int64_t nl = T.cl[1] * cap + nc;
        gstore(B.ent + nl, make_double4(np.x, np.y, np.z, pack_meta(T.sp, (int32_t)T.idx)));
        gstore(B.count + (T.cl[1]), nc + 1);
        gstore(B.pos + T.idx, make_double4(np.x, np.y, np.z, pack_meta(T.sp, (int32_t)nl)));
        if (nc + 1 > maxc) maxc = nc + 1;
        return GCMC_OK;
    }
    if (T.type == GCMC_MOVE_INSERT) {
        if (n >= B.max_n) return GCMC_ERR_CAPACITY;
        const int32_t nc = gload(B.count + (T.cl[0]));
        if (nc >= cap) return GCMC_ERR_CELL_OVERFLOW;
        const int64_t nl = T.cl[0] * cap + nc;
        gstore(B.ent + nl, make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(T.sp, (int32_t)n)));
        gstore(B.count + (T.cl[0]), nc + 1);
        gstore(B.pos + n, make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(T.sp, (int32_t)nl)));
        if (nc + 1 > maxc) maxc = nc + 1;
        return GCMC_OK;
    }
    // deletion: drop the entry, then particle n-1 takes index idx
    const int64_t loc = meta_low(T.meta);
    remove_entry(B, T.cl[0], loc);
    if (T.idx != n - 1) {
        const double4 last = gload(B.pos + (n - 1));
        gstore(B.pos + T.idx, last);
        const int64_t l2 = meta_low(last.w);
        gstore_w(B.ent + l2, pack_meta(meta_species(last.w), (int32_t)T.idx));
    }
    return GCMC_OK;
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
    const double4 pi = gload(B.pos + T.idx);
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

// A register copy of the descriptor fields the chain uses (single species),
// every field passed through readfirstlane so it stays in scalar registers.
__device__ __forceinline__ DevBox hot_copy(const DevBox& G) {
    DevBox B;
    B.pos = unip(G.pos);
    B.ent = unip(G.ent);
    B.count = unip(G.count);
    B.st = unip(G.st);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        B.L[a] = unid(G.L[a]);
        B.hL[a] = unid(G.hL[a]);
        B.invS[a] = unid(G.invS[a]);
        B.M[a] = uni(G.M[a]);
        B.span[a] = uni(G.span[a]);
        B.k[a] = uni(G.k[a]);
        B.full[a] = uni(G.full[a]);
    }
    B.cap = uni(G.cap);
    B.ns = uni(G.ns);
    B.ncells = uni64(G.ncells);
    B.max_n = uni64(G.max_n);
    B.rc2 = unid(G.rc2);
    B.beta = unid(G.beta);
    B.mu = unid(G.mu);
    B.lambda3 = unid(G.lambda3);
    B.max_disp = unid(G.max_disp);
    B.p_disp = unid(G.p_disp);
    B.V = unid(G.V);
    B.eps4[0] = unid(G.eps4[0]);
    B.sig2[0] = unid(G.sig2[0]);
    B.tailK[0] = unid(G.tailK[0]);
    B.ptailK[0] = unid(G.ptailK[0]);
    B.seed = (uint64_t)uni64((int64_t)G.seed);
    B.box_id = (uint32_t)uni((int32_t)G.box_id);
    B.nstencil = uni(G.nstencil);
    B.wait_limit = uni(G.wait_limit);
    B.stab = unip(G.stab);
    return B;
}

}  // namespace gcmc
