// Evaluation of one chain move against the current state by one wavefront,
// shared by the speculative kernels (rounds of W moves, and the pipeline of a
// committer and evaluators).  The wavefront computes the Philox draws of the
// moves that precede its move and are not yet decided (lane 4j + b: block b
// of the j-th of them), counts the insertions (I) and deletions (D) among them
// (N at the move's decision lies in [N - D, N + I]), and picks at the N
// expected from the chain's running acceptance rates; then it loads the
// counters of its stencil cells (one lane per cell), prefix-sums them, maps
// each flattened candidate to its cell through an owner table in LDS, loads
// exactly the candidates' records and reduces the pair sums.
//
// Stencils of more than 32 cells (microcells smaller than the cutoff, whose
// stencils of 2k+1 cells per axis are pruned of the cells beyond it) take a
// second path: the cells are loaded in groups of 64, one lane per cell (all
// groups' counters in one memory round trip), prefix-summed across the
// groups, and the flattened candidates' record indices are written to an LDS
// table that is filled and consumed in windows, so a move may have any number
// of candidates.
#pragma once
#include "trial.h"

namespace gcmc {

constexpr int kSpecOwn = 8192;       // flattened candidates per wavefront (owner table bytes)
constexpr int kSpecRecWin = kSpecOwn / 4;   // record indices per window of the microcell path (same bytes)
constexpr int kSpecGroups = 16;      // groups of 64 stencil cells: stencils of up to 512 cells (two for a displacement)
constexpr int kSpecMaxStencil = kSpecGroups * kWave / 2;
constexpr int kSpecGroupsSmall = 4;  // the instantiation for stencils of up to 128 cells (fewer registers)

struct SpecRec {
    double dUp, lnA, u2, dWp;   // pair energy change, ln A, pick draw, pair virial change
    double p0[3], p1[3];
    double4 rec, elast;
    int64_t idx;
    int32_t type, flags, two, pad;
    int32_t c0[3], c1[3];
    int32_t cl0, cl1, cnt0, cnt1;
    int32_t cand, evals, incut, pad2;
};

// Inclusive prefix sum over the wavefront's lanes (DPP row shifts, then the
// row broadcasts of gfx9 carry each row's total into the next rows).
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

__device__ __forceinline__ int spec_type(const DevBox& B, const U8& u) {
    return (u.u[0] < B.p_disp) ? GCMC_MOVE_DISPLACE : ((u.u[1] < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
}

__device__ __forceinline__ int64_t spec_pick(double u, int64_t n) {
    int64_t i = (int64_t)floor(u * (double)n);
    return i > n - 1 ? n - 1 : i;
}

__device__ __forceinline__ int32_t spec_axis_cell(double x, double invS, int32_t M) {
    return __builtin_amdgcn_readfirstlane(axis_cell(x, invS, M));
}

// Is cell (x, y, z) inside the stencil of centre cell c?
__device__ __forceinline__ bool in_stencil(const DevBox& B, int32_t x, int32_t y, int32_t z, const int32_t* c) {
    const int32_t v[3] = {x, y, z};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int32_t d = v[a] - c[a];
        d = d < 0 ? -d : d;
        const int32_t e = B.M[a] - d;
        d = e < d ? e : d;
        in = in && (B.full[a] || d <= B.k[a]);
    }
    return in;
}

// One candidate record against the move's position(s): energy and virial sums.
__device__ __forceinline__ void spec_pair(const DevBox& B, int type, int two, bool second, const double* p0,
                                          const double* p1, const double4& e, double& sa, double& sb, double& wa,
                                          double& wb, int32_t& n_eval, int64_t& incut) {
    if (type != GCMC_MOVE_DISPLACE) {
        sa += pair_uw<false>(B, p0, 0, e, incut, wa);
        n_eval += 1;
    } else if (!two) {
        sa += pair_uw<false>(B, p0, 0, e, incut, wa);
        sb += pair_uw<false>(B, p1, 0, e, incut, wb);
        n_eval += 2;
    } else if (second) {
        sb += pair_uw<false>(B, p1, 0, e, incut, wb);
        n_eval += 1;
    } else {
        sa += pair_uw<false>(B, p0, 0, e, incut, wa);
        n_eval += 1;
    }
}

// Wavefront k evaluates move ctr_round + k against the current state.  NG:
// 0 for the 32-cell path, else the number of groups of 64 stencil cells the
// microcell path provides (see above).
template <int CR, int NG>
__device__ __forceinline__ void spec_eval(const DevBox& B, const uint32_t* tab, const int32_t* offs, void* ownbuf,
                                          uint64_t ctr_round, int k, int64_t N, bool no_full, double a_ins,
                                          double a_del, SpecRec* out) {
    const int lane = threadIdx.x & (kWave - 1);
    // draws of the round's moves: lane 4j + b computes Philox block b of move ctr_round + j
    double ua, ub;
    {
        const uint64_t c = ctr_round + (uint64_t)(lane >> 2);
        uint32_t c0 = (uint32_t)c, c1 = (uint32_t)(c >> 32), c2 = B.box_id, c3 = (uint32_t)(lane & 3);
        philox_block(c0, c1, c2, c3, (uint32_t)B.seed, (uint32_t)(B.seed >> 32));
        ua = to_unit(c0, c1);
        ub = to_unit(c2, c3);
    }
    U8 u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        u.u[2 * q] = read_lane(ua, 4 * k + q);
        u.u[2 * q + 1] = read_lane(ub, 4 * k + q);
    }
    const int type = __builtin_amdgcn_readfirstlane(spec_type(B, u));
    // insertions (I) and deletions (D) among the earlier moves of the round: N at this
    // move's commit lies in [N - D, N + I]
    const int tj = (ua < B.p_disp) ? GCMC_MOVE_DISPLACE : ((ub < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
    const bool earlier = (lane & 3) == 0 && (lane >> 2) < k;
    const int64_t D = __popcll(__ballot(earlier && tj == GCMC_MOVE_DELETE));
    const int64_t I = __popcll(__ballot(earlier && tj == GCMC_MOVE_INSERT));
    if (type != GCMC_MOVE_INSERT && N == 0) {
        if (lane == 0) {
            out->type = type;
            out->flags = 1;
            out->lnA = 0.0;
            out->u2 = u.u[2];
            out->cand = out->evals = out->incut = 0;
        }
        return;
    }
    int64_t idx = -1;
    double4 rec = make_double4(0, 0, 0, 0);
    double p0[3], p1[3];
    if (type == GCMC_MOVE_INSERT) {
#pragma unroll
        for (int a = 0; a < 3; ++a) p0[a] = wrap_into_box(B.L[a] * u.u[4 + a], B.L[a]);
    } else {
        // the pick at the N expected at commit from the running acceptance rates
        const int64_t n_lo = (N - D) > 1 ? (N - D) : 1, n_hi = N + I;
        int64_t n_c = (int64_t)floor((double)N + (double)I * a_ins - (double)D * a_del + 0.5);
        n_c = uni64(n_c < n_lo ? n_lo : (n_c > n_hi ? n_hi : n_c));
        idx = spec_pick(u.u[2], n_c);
        rec = gload(B.pos + idx);
        p0[0] = rec.x; p0[1] = rec.y; p0[2] = rec.z;
    }
    int32_t c0[3], c1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c0[a] = spec_axis_cell(p0[a], B.invS[a], B.M[a]);
    const int32_t cl0 = (c0[2] * B.M[1] + c0[1]) * B.M[0] + c0[0];
    int32_t cl1 = cl0;
    int same = 1;
    if (type == GCMC_MOVE_DISPLACE) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p1[a] = wrap_into_box(p0[a] + B.max_disp * (2.0 * u.u[4 + a] - 1.0), B.L[a]);
            c1[a] = spec_axis_cell(p1[a], B.invS[a], B.M[a]);
        }
        cl1 = (c1[2] * B.M[1] + c1[1]) * B.M[0] + c1[0];
        same = __builtin_amdgcn_readfirstlane(cl1 == cl0 ? 1 : 0);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p1[a] = p0[a];
            c1[a] = c0[a];
        }
    }
    const int two = (type == GCMC_MOVE_DISPLACE && !same) ? 1 : 0;
    const int nst = B.nstencil;
    const int ncs = two ? 2 * nst : nst;
    // ---- counters of the stencil cells, one lane per cell
    const bool fast = __builtin_amdgcn_readfirstlane(
                          (no_full && c0[0] >= B.k[0] && c0[0] <= B.M[0] - 1 - B.k[0] && c0[1] >= B.k[1] &&
                           c0[1] <= B.M[1] - 1 - B.k[1] && c0[2] >= B.k[2] && c0[2] <= B.M[2] - 1 - B.k[2] &&
                           (!two || (c1[0] >= B.k[0] && c1[0] <= B.M[0] - 1 - B.k[0] && c1[1] >= B.k[1] &&
                                     c1[1] <= B.M[1] - 1 - B.k[1] && c1[2] >= B.k[2] &&
                                     c1[2] <= B.M[2] - 1 - B.k[2])))
                              ? 1
                              : 0) != 0;
    int32_t cnt0 = 0, cnt1 = 0;
    double4 elast = make_double4(0, 0, 0, 0);
    const int32_t excl = (int32_t)idx;
    double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
    int32_t n_cand = 0, n_eval = 0, n_in = 0;
    int64_t incut = 0;
    if constexpr (NG == 0) {
        const int wh = lane >= nst ? 1 : 0;
        const int t = lane - wh * nst;
        const bool cell_lane = lane < ncs;
        int32_t cell = cl0;
        if (cell_lane) {
            if (fast) {
                cell = (wh ? cl1 : cl0) + offs[t];
            } else {
                cell = (int32_t)stencil_cell(B, tab[t], wh ? c1[0] : c0[0], wh ? c1[1] : c0[1], wh ? c1[2] : c0[2]);
            }
        }
        const int32_t cnt = cell_lane ? gload(B.count + cell) : 0;
        const int32_t incl = wave_incl_scan(cnt);
        const int32_t pre = incl - cnt;
        const int32_t total = __builtin_amdgcn_readlane(incl, 63);
        // lanes of the two centre cells (each appears once in its stencil)
        const int tc = (int)__builtin_ctzll(__ballot(cell_lane && !wh && cell == cl0));
        const int tc1 = two ? (int)__builtin_ctzll(__ballot(cell_lane && wh && cell == cl1)) : tc;
        cnt0 = __builtin_amdgcn_readlane(cnt, tc);
        cnt1 = __builtin_amdgcn_readlane(cnt, tc1);
        // ---- owner of each flattened candidate
        uint8_t* own = static_cast<uint8_t*>(ownbuf);
        const int kmax = wave_max_i32_uniform(cnt);
        for (int k = 0; k < kmax; ++k)
            if (k < cnt) own[pre + k] = (uint8_t)lane;
        const int32_t cellbase = cell * B.cap - pre;   // record index of flattened candidate q: q + cellbase[owner]
        __builtin_amdgcn_wave_barrier();
        // last entry of the old centre cell (removal by swap-with-last)
        if (cnt0 > 0) elast = gload(B.ent + ((size_t)(uint32_t)cl0 * (uint32_t)B.cap + (cnt0 - 1)));
        // ---- candidates
        for (int base = 0; base < total; base += kWave * CR) {
            double4 e[CR];
            int32_t wsel[CR];
            bool ok[CR];
    #pragma unroll
            for (int r = 0; r < CR; ++r) {
                const int q = base + r * kWave + lane;
                ok[r] = q < total;
                const int j = ok[r] ? own[q] : 0;
                const int32_t cb = __shfl(cellbase, j, kWave);
                wsel[r] = j >= nst ? 1 : 0;
                e[r] = gload(B.ent + (size_t)(uint32_t)(ok[r] ? cb + q : cl0 * B.cap));
            }
    #pragma unroll
            for (int r = 0; r < CR; ++r) {
                if (ok[r] && meta_low(e[r].w) != excl) {
                    n_cand += 1;
                    if (type != GCMC_MOVE_DISPLACE) {
                        sa += pair_uw<false>(B, p0, 0, e[r], incut, wa);
                        n_eval += 1;
                    } else if (!two) {
                        sa += pair_uw<false>(B, p0, 0, e[r], incut, wa);
                        sb += pair_uw<false>(B, p1, 0, e[r], incut, wb);
                        n_eval += 2;
                    } else if (wsel[r]) {
                        sb += pair_uw<false>(B, p1, 0, e[r], incut, wb);
                        n_eval += 1;
                    } else {
                        sa += pair_uw<false>(B, p0, 0, e[r], incut, wa);
                        n_eval += 1;
                    }
                }
            }
        }

    } else {
        // ---- microcell stencils: groups of 64 cells, one lane per cell
        const int G = (ncs + kWave - 1) / kWave;
        int32_t cellg[NG], cntg[NG], preg[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            cellg[g] = cl0;
            cntg[g] = 0;
            if (g < G) {
                const int f = g * kWave + lane;
                const int wh = f >= nst ? 1 : 0;
                const int t = f - wh * nst;
                if (f < ncs)
                    cellg[g] = fast ? (wh ? cl1 : cl0) + offs[t]
                                    : (int32_t)stencil_cell(B, tab[t], wh ? c1[0] : c0[0], wh ? c1[1] : c0[1],
                                                            wh ? c1[2] : c0[2]);
                cntg[g] = f < ncs ? gload(B.count + cellg[g]) : 0;
            }
        }
        int32_t total = 0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            preg[g] = 0;
            if (g < G) {
                const int f = g * kWave + lane;
                const bool on = f < ncs;
                const int wh = f >= nst ? 1 : 0;
                const int32_t incl = wave_incl_scan(cntg[g]);
                preg[g] = total + incl - cntg[g];
                total += __builtin_amdgcn_readlane(incl, 63);
                // the centre cells (each appears once in its stencil)
                const uint64_t b0 = __ballot(on && !wh && cellg[g] == cl0);
                if (b0) cnt0 = __builtin_amdgcn_readlane(cntg[g], (int)__builtin_ctzll(b0));
                const uint64_t b1 = __ballot(on && wh && cellg[g] == cl1);
                if (b1) cnt1 = __builtin_amdgcn_readlane(cntg[g], (int)__builtin_ctzll(b1));
            }
        }
        if (!two) cnt1 = cnt0;
        if (cnt0 > 0) elast = gload(B.ent + ((size_t)(uint32_t)cl0 * (uint32_t)B.cap + (cnt0 - 1)));
        // ---- record indices of the flattened candidates, window by window (bit 31: second stencil)
        uint32_t* recw = static_cast<uint32_t*>(ownbuf);
        for (int q0 = 0; q0 < total; q0 += kSpecRecWin) {
            const int q1 = (total - q0) < kSpecRecWin ? total : q0 + kSpecRecWin;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (g < G) {
                    const uint32_t second = (g * kWave + lane) >= nst ? 0x80000000u : 0u;
                    const uint32_t rb = (uint32_t)cellg[g] * (uint32_t)B.cap;
                    const int kmax = wave_max_i32_uniform(cntg[g]);
                    for (int kk = 0; kk < kmax; ++kk) {
                        const int q = preg[g] + kk;
                        if (kk < cntg[g] && q >= q0 && q < q1) recw[q - q0] = (rb + (uint32_t)kk) | second;
                    }
                }
            }
            // the indices other lanes of this wavefront wrote, visible to every lane
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
            for (int base = q0; base < q1; base += kWave * CR) {
                double4 e[CR];
                bool ok[CR], sec[CR];
#pragma unroll
                for (int r = 0; r < CR; ++r) {
                    const int q = base + r * kWave + lane;
                    ok[r] = q < q1;
                    const uint32_t v = ok[r] ? recw[q - q0] : (uint32_t)cl0 * (uint32_t)B.cap;
                    sec[r] = (v & 0x80000000u) != 0;
                    e[r] = gload(B.ent + (size_t)(v & 0x7FFFFFFFu));
                }
#pragma unroll
                for (int r = 0; r < CR; ++r) {
                    if (ok[r] && meta_low(e[r].w) != excl) {
                        n_cand += 1;
                        spec_pair(B, type, two, sec[r], p0, p1, e[r], sa, sb, wa, wb, n_eval, incut);
                    }
                }
            }
            // every lane has read this window before the next overwrites it
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
        }
    }
    n_in = (int32_t)incut;
    const double ea = wave_sum_uniform(sa);
    const double eb = (type == GCMC_MOVE_DISPLACE) ? wave_sum_uniform(sb) : 0.0;
    const double dUp = (type == GCMC_MOVE_DISPLACE) ? (eb - ea) : ((type == GCMC_MOVE_INSERT) ? ea : -ea);
    const double va = wave_sum_vec(wa);
    const double vb = (type == GCMC_MOVE_DISPLACE) ? wave_sum_vec(wb) : 0.0;
    const double dWp = (type == GCMC_MOVE_DISPLACE) ? (vb - va) : ((type == GCMC_MOVE_INSERT) ? va : -va);
    // work counters of this evaluation (wave sums)
    n_cand = wave_sum_i32_uniform(n_cand);
    n_eval = wave_sum_i32_uniform(n_eval);
    n_in = wave_sum_i32_uniform(n_in);
    const double lnA = log(u.u[3]);
    if (lane == 0) {
        out->dUp = dUp;
        out->dWp = dWp;
        out->lnA = lnA;
        out->u2 = u.u[2];
        out->type = type;
        out->flags = 0;
        out->two = two;
        out->idx = idx;
        out->rec = rec;
        out->elast = elast;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            out->p0[a] = p0[a];
            out->p1[a] = p1[a];
            out->c0[a] = c0[a];
            out->c1[a] = c1[a];
        }
        out->cl0 = cl0;
        out->cl1 = cl1;
        out->cnt0 = cnt0;
        out->cnt1 = cnt1;
        out->cand = n_cand;
        out->evals = n_eval;
        out->incut = n_in;
    }
}

}  // namespace gcmc
