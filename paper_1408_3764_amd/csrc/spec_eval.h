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
//
// Only about one candidate in seven lies inside the cutoff, and a wavefront
// executes the Lennard-Jones arithmetic whenever one of its lanes needs it.
// So the candidate pass only computes squared distances; the in-cutoff ones
// are queued in a per-wavefront ring in LDS (the sign bit marks the second
// position of a displacement) and the pair energies and virials are
// evaluated 64 at a time, one per lane.
//
// The draws (move type, pick, position, ln A) come either from a ring of
// draws in LDS that the round kernel fills once per round for the moves it may
// take next, or are computed here (the pipelined kernel).
#pragma once
#include "trial.h"

namespace gcmc {

constexpr int kSpecOwn = 8192;       // flattened candidates per wavefront (owner table bytes)
constexpr int kSpecRecWin = kSpecOwn / 4;   // record indices per window of the microcell path (same bytes)
// 32-bit words of a wavefront's owner buffer: the 32-cell path keeps 64 cell bases and one
// start mask per 64 flattened candidates; the microcell path a window of record indices
constexpr int spec_own_words(int ng) { return ng ? kSpecRecWin : kWave + 2 * (kSpecOwn / 64); }
constexpr int kSpecGroups = 16;      // groups of 64 stencil cells: stencils of up to 512 cells (two for a displacement)
constexpr int kSpecMaxStencil = kSpecGroups * kWave / 2;
constexpr int kSpecGroupsSmall = 4;  // the instantiation for stencils of up to 128 cells (fewer registers)
constexpr int kPairRing = 128;       // queued in-cutoff pairs per wavefront (a power of two, >= 2 x 64)

// Draws of the moves a round may take, one slot per move (slot = move counter
// mod RING, RING a power of two): move type, pick draw, ln A, and the three
// position draws (insertion point, or the displacement).
template <int RING>
struct DrawRing {
    double u2[RING], u7[RING], lnA[RING], px[RING], py[RING], pz[RING];
    int32_t type[RING];
};

// Philox block `b` of move `ctr` into its ring slot (one lane per block:
// block 0 gives the type, 1 the pick draw and ln A, 2 and 3 the position
// draws and the pick fields).
template <int RING>
__device__ __forceinline__ void draw_block(const DevBox& B, DrawRing<RING>* dr, uint64_t ctr, int b) {
    uint32_t c0 = (uint32_t)ctr, c1 = (uint32_t)(ctr >> 32), c2 = B.box_id, c3 = (uint32_t)b;
    philox_block(c0, c1, c2, c3, (uint32_t)B.seed, (uint32_t)(B.seed >> 32));
    const double ua = to_unit(c0, c1), ub = to_unit(c2, c3);
    const int s = (int)(ctr & (uint64_t)(RING - 1));
    if (b == 0) {
        dr->type[s] = (ua < B.p_disp) ? GCMC_MOVE_DISPLACE : ((ub < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
    } else if (b == 1) {
        dr->u2[s] = ua;
        dr->lnA[s] = log(ub);
    } else if (b == 2) {
        dr->px[s] = ua;
        dr->py[s] = ub;
    } else {
        dr->pz[s] = ua;
        dr->u7[s] = ub;
    }
}

// Per-wavefront queue of in-cutoff squared distances.  push: the lanes with
// `in` append v (ballot order); drain: lane l takes entry head + l of the
// next `cnt` and adds its pair energy and virial to the first position's sums,
// or the second's when v carries the sign bit.
__device__ __forceinline__ void pair_push(double* q, uint32_t& tail, bool in, double v) {
    const uint64_t m = __ballot(in);
    if (in) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        q[(tail + below) & (kPairRing - 1)] = v;
    }
    tail += (uint32_t)__builtin_popcountll(m);
}

__device__ __forceinline__ void pair_drain(const DevBox& B, const double* q, uint32_t head, uint32_t cnt, double& sa,
                                           double& sb, double& wa, double& wb) {
    // the entries other lanes wrote, visible to every lane
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (lane < cnt) {
        const double v = q[(head + lane) & (kPairRing - 1)];
        const bool second = __builtin_signbit(v);
        const double r2 = second ? -v : v;
        double w = 0.0;
        const double u = lj_uw_from_r2(r2, B.rc2, B.eps4[0], B.sig2[0], w);
        if (second) {
            sb += u;
            wb += w;
        } else {
            sa += u;
            wa += w;
        }
    }
    // every lane has read its entry before later pushes reuse the slots
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
}

// Squared distances of one candidate record to the move's position(s),
// queued when inside the cutoff (counts of evaluated and in-cutoff pairs kept
// per lane).
// Squared distance of a candidate to a position; the minimum image only where
// the stencil may cross a periodic face (wrap false: every candidate lies
// within (k + 1) cells of the position along each axis, at least half a cell
// short of L/2, where the minimum image returns the difference unchanged, bit
// for bit).
__device__ __forceinline__ double spec_dist2(const DevBox& B, const double* p, const double3& e, bool wrap) {
    double dx = e.x - p[0], dy = e.y - p[1], dz = e.z - p[2];
    if (wrap) {
        dx = nearest_image(dx, B.L[0], B.hL[0]);
        dy = nearest_image(dy, B.L[1], B.hL[1]);
        dz = nearest_image(dz, B.L[2], B.hL[2]);
    }
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ void spec_pair_queue(const DevBox& B, int type, int two, bool valid, bool second,
                                                const double* p0, const double* p1, const double3& e, bool wrap,
                                                double* q, uint32_t& head, uint32_t& tail, double& sa, double& sb,
                                                double& wa, double& wb, int32_t& n_eval, int64_t& incut) {
    const bool disp = type == GCMC_MOVE_DISPLACE;
    // the first position: every move but the second stencil of a displacement that leaves its cell
    const bool use0 = valid && !(disp && two && second);
    const bool use1 = valid && disp && (!two || second);
    double r2a = 0.0, r2b = 0.0;
    if (use0) r2a = spec_dist2(B, p0, e, wrap);
    const bool in0 = use0 && r2a < B.rc2;
    n_eval += use0 ? 1 : 0;
    incut += in0 ? 1 : 0;
    pair_push(q, tail, in0, r2a);
    if (tail - head >= (uint32_t)kWave) {
        pair_drain(B, q, head, kWave, sa, sb, wa, wb);
        head += kWave;
    }
    if (disp) {
        if (use1) r2b = spec_dist2(B, p1, e, wrap);
        const bool in1 = use1 && r2b < B.rc2;
        n_eval += use1 ? 1 : 0;
        incut += in1 ? 1 : 0;
        pair_push(q, tail, in1, -r2b);
        if (tail - head >= (uint32_t)kWave) {
            pair_drain(B, q, head, kWave, sa, sb, wa, wb);
            head += kWave;
        }
    }
}

// The coordinates of a 32-byte record (its fourth word, the id, is not
// needed: a move's own particle is excluded by its slot).
__device__ __forceinline__ double3 gload_xyz(const double4* p) {
    typedef double gcmc_d2v __attribute__((ext_vector_type(2)));
    const GCMC_GLOBAL_AS double* q = (const GCMC_GLOBAL_AS double*)p;
    const gcmc_d2v xy = *(const GCMC_GLOBAL_AS gcmc_d2v*)q;
    return make_double3(xy.x, xy.y, q[2]);
}

struct SpecRec {
    // what the in-order commit reads for every move, first
    int32_t type, flags;
    uint32_t pickmask, okmask;   // bit o: the pick still valid / the move accepted at N = N_round - (W - 1) + o
    int64_t idx;
    int32_t c0[3], c1[3];
    // what it reads for an accepted move
    int32_t two, cnt0, cnt1, cl0, cl1, pad;
    double dUp, dWp, lnA, u2, u7;   // pair energy change, pair virial change, ln A, pick draws
    double p0[3], p1[3];
    double4 rec, elast;
    int32_t cand, evals, incut, pad2;
};

// The values of an evaluation the round kernel decides with in advance.
struct SpecKey {
    int32_t type, flags;
    int64_t idx;
    double u2, u7, lnA, dUp;
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

__device__ __forceinline__ int64_t spec_pick(double u2, double u7, int64_t n) { return pick_particle(u2, u7, n); }

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

// The caller's work that needs only the move's type, draws and pick, run by
// the evaluation while the picked record is being loaded (none by default).
struct SpecNoEarly {
    __device__ __forceinline__ void operator()(int, double, double, int64_t) const {}
};

// Wavefront k evaluates move ctr_round + k against the current state.  NG:
// 0 for the 32-cell path, else the number of groups of 64 stencil cells the
// microcell path provides (see above).  RING > 0: the draws come from `dr`
// (the moves ctr_round .. ctr_round + k must be in it); RING = 0: computed
// here, for k < 16.  pq: this wavefront's pair queue (kPairRing doubles of
// LDS).
template <int CR, int NG, int RING, typename Early = SpecNoEarly>
__device__ __forceinline__ void spec_eval(const DevBox& B, const uint32_t* tab, const int32_t* offs, void* ownbuf,
                                          double* pq, const DrawRing<RING>* dr, uint64_t ctr_round, int k, int64_t N,
                                          bool no_full, double a_ins, double a_del, SpecRec* out, SpecKey& key,
                                          const Early& early = Early()) {
    const int lane = threadIdx.x & (kWave - 1);
    int type;
    double u2, u7, lnA, ux, uy, uz;
    int64_t D, I;
    if constexpr (RING > 0) {
        // the round's draws from the ring; lane j < k reads the type of the j-th earlier move
        const int s = (int)((ctr_round + (uint64_t)k) & (uint64_t)(RING - 1));
        type = uni(dr->type[s]);
        u2 = dr->u2[s];
        u7 = dr->u7[s];
        lnA = dr->lnA[s];
        ux = dr->px[s];
        uy = dr->py[s];
        uz = dr->pz[s];
        const int tj = lane < k ? dr->type[(int)((ctr_round + (uint64_t)lane) & (uint64_t)(RING - 1))] : -1;
        D = __popcll(__ballot(tj == GCMC_MOVE_DELETE));
        I = __popcll(__ballot(tj == GCMC_MOVE_INSERT));
    } else {
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
        type = __builtin_amdgcn_readfirstlane(spec_type(B, u));
        u2 = u.u[2];
        u7 = u.u[7];
        lnA = log(u.u[3]);
        ux = u.u[4];
        uy = u.u[5];
        uz = u.u[6];
        // insertions (I) and deletions (D) among the earlier moves of the round: N at this
        // move's commit lies in [N - D, N + I]
        const int tj = (ua < B.p_disp) ? GCMC_MOVE_DISPLACE : ((ub < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
        const bool earlier = (lane & 3) == 0 && (lane >> 2) < k;
        D = __popcll(__ballot(earlier && tj == GCMC_MOVE_DELETE));
        I = __popcll(__ballot(earlier && tj == GCMC_MOVE_INSERT));
    }
    const double ud[3] = {ux, uy, uz};
    key.type = type;
    key.flags = 0;
    key.u2 = u2;
    key.u7 = u7;
    key.lnA = lnA;
    key.idx = -1;
    key.dUp = 0.0;
    if (type != GCMC_MOVE_INSERT && N == 0) {
        key.flags = 1;
        if (lane == 0) {
            out->type = type;
            out->flags = 1;
            out->lnA = 0.0;
            out->u2 = u2;
            out->u7 = u7;
            out->cand = out->evals = out->incut = 0;
        }
        return;
    }
    int64_t idx = -1;
    double4 rec = make_double4(0, 0, 0, 0);
    double p0[3], p1[3];
    if (type == GCMC_MOVE_INSERT) {
#pragma unroll
        for (int a = 0; a < 3; ++a) p0[a] = wrap_into_box(B.L[a] * ud[a], B.L[a]);
        early(type, u2, u7, idx);
    } else {
        // the pick at the N expected at commit from the running acceptance rates
        const int64_t n_lo = (N - D) > 1 ? (N - D) : 1, n_hi = N + I;
        int64_t n_c = (int64_t)floor((double)N + (double)I * a_ins - (double)D * a_del + 0.5);
        n_c = uni64(n_c < n_lo ? n_lo : (n_c > n_hi ? n_hi : n_c));
        idx = spec_pick(u2, u7, n_c);
        rec = gload(B.pos + idx);
        early(type, u2, u7, idx);   // the caller's work that needs only the pick, while the record loads
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
            p1[a] = wrap_into_box(p0[a] + B.max_disp * (2.0 * ud[a] - 1.0), B.L[a]);
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
    // candidates need the minimum image unless the stencils stay inside the box with room to spare
    const bool wrap = !(fast && B.M[0] >= 2 * B.k[0] + 3 && B.M[1] >= 2 * B.k[1] + 3 && B.M[2] >= 2 * B.k[2] + 3);
    int32_t cnt0 = 0, cnt1 = 0;
    double4 elast = make_double4(0, 0, 0, 0);
    // the slot of the moving particle's own record in the cell array (never a candidate of itself)
    const int32_t excl_slot = type == GCMC_MOVE_INSERT ? -1 : meta_low(rec.w);
    double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
    int32_t n_cand = 0, n_eval = 0, n_in = 0;
    int64_t incut = 0;
    uint32_t qhead = 0, qtail = 0;   // the in-cutoff pair queue (wave-uniform counters)
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
        // ---- owner of each flattened candidate: the nonempty cells, in lane order, are numbered
        // k = 0, 1, ...; cbk[k] = the cell's record index minus its first flattened position,
        // and bit q of the row masks marks a flattened position q where a nonempty cell begins,
        // so the owner of q is the number of marks at or below q, minus one
        uint32_t* cbk = static_cast<uint32_t*>(ownbuf);                // [64]
        uint64_t* smask = reinterpret_cast<uint64_t*>(cbk + kWave);   // [kSpecOwn / 64]
        const int nrows = (total + kWave - 1) / kWave;
        for (int r = lane; r < nrows; r += kWave) smask[r] = 0;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
        {
            const bool nonempty = cnt > 0;
            const uint64_t nzm = __ballot(nonempty);
            if (nonempty) {
                const uint32_t k = __builtin_amdgcn_mbcnt_hi((uint32_t)(nzm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)nzm, 0u));
                cbk[k] = (uint32_t)(cell * B.cap - pre);
                __hip_atomic_fetch_or(&smask[pre >> 6], 1ull << (pre & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        }
        const int32_t first2 = __builtin_amdgcn_readlane(incl, nst - 1);   // flattened start of the second stencil
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
        uint32_t starts = 0;   // nonempty cells beginning before the current row (wave-uniform)
        // last entry of the old centre cell (removal by swap-with-last)
        if (cnt0 > 0) elast = gload(B.ent + ((size_t)(uint32_t)cl0 * (uint32_t)B.cap + (cnt0 - 1)));
        // ---- candidates
        for (int base = 0; base < total; base += kWave * CR) {
            double3 e[CR];
            int32_t wsel[CR];
            bool ok[CR];
    #pragma unroll
            for (int r = 0; r < CR; ++r) {
                const int q = base + r * kWave + lane;
                const int row = (base >> 6) + r;
                const uint64_t m = row < nrows ? smask[row] : 0;
                const uint32_t k = starts + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) +
                                   (uint32_t)((m >> lane) & 1ull) - 1u;
                starts += (uint32_t)__builtin_popcountll(m);
                const int32_t cb = q < total ? (int32_t)cbk[k & (kWave - 1)] : 0;
                const int32_t ri = q < total ? cb + q : cl0 * B.cap;
                ok[r] = q < total && ri != excl_slot;
                wsel[r] = (nst < ncs && q >= first2) ? 1 : 0;
                e[r] = gload_xyz(B.ent + (size_t)(uint32_t)ri);
            }
    #pragma unroll
            for (int r = 0; r < CR; ++r) {
                // rows past the last candidate hold nothing for any lane (wave-uniform)
                if (base + r * kWave >= total) break;
                const bool valid = ok[r];
                n_cand += valid ? 1 : 0;
                spec_pair_queue(B, type, two, valid, wsel[r] != 0, p0, p1, e[r], wrap, pq, qhead, qtail, sa, sb, wa,
                                wb, n_eval, incut);
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
                double3 e[CR];
                bool ok[CR], sec[CR];
#pragma unroll
                for (int r = 0; r < CR; ++r) {
                    const int q = base + r * kWave + lane;
                    const uint32_t v = q < q1 ? recw[q - q0] : (uint32_t)cl0 * (uint32_t)B.cap;
                    sec[r] = (v & 0x80000000u) != 0;
                    ok[r] = q < q1 && (int32_t)(v & 0x7FFFFFFFu) != excl_slot;
                    e[r] = gload_xyz(B.ent + (size_t)(v & 0x7FFFFFFFu));
                }
#pragma unroll
                for (int r = 0; r < CR; ++r) {
                    // rows past the window's last candidate hold nothing for any lane (wave-uniform)
                    if (base + r * kWave >= q1) break;
                    const bool valid = ok[r];
                    n_cand += valid ? 1 : 0;
                    spec_pair_queue(B, type, two, valid, sec[r], p0, p1, e[r], wrap, pq, qhead, qtail, sa, sb, wa,
                                    wb, n_eval, incut);
                }
            }
            // every lane has read this window before the next overwrites it
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
        }
    }
    // the pairs still queued
    if (qtail != qhead) pair_drain(B, pq, qhead, qtail - qhead, sa, sb, wa, wb);
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
    key.idx = idx;
    key.dUp = dUp;
    if (lane == 0) {
        out->dUp = dUp;
        out->dWp = dWp;
        out->lnA = lnA;
        out->u2 = u2;
        out->u7 = u7;
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
