// Total energy, the all-pairs (no cell list) energy path, and the gradient.
//
// Total energy over the cell list: one lane per particle, the particles taken
// in cell-major order (cell by cell, slot by slot: the order comes from an
// exclusive scan of the cell counters), so no lane idles on an empty slot and
// the lanes of one wavefront belong to a few consecutive cells.  Each lane
// walks the stencil of its own cell and sums its pair energies e_i in stencil
// order, candidate order; U_pair = (1/2) sum e_i (Sec. 3.1.1 computes each
// unique pair once; here each pair is met from both ends, which needs no
// atomics), workgroup partials are summed by one more workgroup in a fixed
// order.
//
// The all-pairs path (Algorithms 3 and 4 without a cell list) streams the
// particle records in chunks, one chunk per workgroup, with the same
// fixed-order second pass.
#include "gcmc_internal.h"

namespace gcmc {

constexpr int kBlk = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    const int nw = blockDim.x / kWave;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// Constants of an energy pass held in registers for the whole kernel (read
// once from the descriptor: the compiler would otherwise reload them from
// memory inside the candidate loop), the species tables in LDS.
struct PassConst {
    double L[3], hL[3], rc2, e4, s2;
};

__device__ __forceinline__ PassConst pass_const(const DevBox& B) {
    PassConst c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.L[a] = unid(B.L[a]);
        c.hL[a] = unid(B.hL[a]);
    }
    c.rc2 = unid(B.rc2);
    c.e4 = unid(B.eps4[0]);
    c.s2 = unid(B.sig2[0]);
    return c;
}

// Squared minimum-image distance with the pass constants (the same
// operations, in the same order, as dist2).
__device__ __forceinline__ double pass_dist2(const PassConst& K, double px, double py, double pz, double qx, double qy,
                                             double qz) {
    const double dx = nearest_image(qx - px, K.L[0], K.hL[0]);
    const double dy = nearest_image(qy - py, K.L[1], K.hL[1]);
    const double dz = nearest_image(qz - pz, K.L[2], K.hL[2]);
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ void load_species_tables(const DevBox& B, double* e4, double* s2) {
    if (threadIdx.x < kMaxSpecies * kMaxSpecies) {
        e4[threadIdx.x] = B.eps4[threadIdx.x];
        s2[threadIdx.x] = B.sig2[threadIdx.x];
    }
}

__device__ __forceinline__ void cell_coords(const DevBox& B, int64_t c, int32_t& cx, int32_t& cy, int32_t& cz) {
    cx = (int32_t)(c % B.M[0]);
    const int64_t r = c / B.M[0];
    cy = (int32_t)(r % B.M[1]);
    cz = (int32_t)(r / B.M[1]);
}

// ------------------------------------------------ particles in cell order
// home[off[c] + k] = c * cap + k for k < count[c]: the cell entry of every
// particle, cell by cell.  off is the exclusive scan of the counters, taken in
// blocks of kScanCells cells (bsum: the blocks' totals, then their exclusive
// scan), so the order is a function of the configuration alone.
constexpr int kScanPer = 4;
constexpr int kScanCells = kBlk * kScanPer;

__global__ __launch_bounds__(kBlk) void k_scan_cells(const int32_t* __restrict__ count, int64_t ncells,
                                                      int32_t* off, int32_t* bsum) {
    __shared__ int32_t sh[kBlk];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanCells + (int64_t)tid * kScanPer;
    int32_t v[kScanPer];
    int32_t tot = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        v[u] = base + u < ncells ? count[base + u] : 0;
        tot += v[u];
    }
    sh[tid] = tot;
    __syncthreads();
    for (int d = 1; d < kBlk; d <<= 1) {
        const int32_t t = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    int32_t run = sh[tid] - tot;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        if (base + u < ncells) off[base + u] = run;
        run += v[u];
    }
    if (tid == kBlk - 1) bsum[blockIdx.x] = sh[tid];
}

// Exclusive scan of the block totals, in place (one workgroup; each thread
// takes a contiguous run of blocks).
__global__ __launch_bounds__(kBlk) void k_scan_sums(int32_t* bsum, int64_t nb) {
    __shared__ int32_t sh[kBlk];
    const int tid = threadIdx.x;
    const int64_t per = (nb + kBlk - 1) / kBlk;
    const int64_t b0 = (int64_t)tid * per;
    int32_t tot = 0;
    for (int64_t b = b0; b < b0 + per && b < nb; ++b) tot += bsum[b];
    sh[tid] = tot;
    __syncthreads();
    for (int d = 1; d < kBlk; d <<= 1) {
        const int32_t t = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    int32_t run = sh[tid] - tot;
    for (int64_t b = b0; b < b0 + per && b < nb; ++b) {
        const int32_t t = bsum[b];
        bsum[b] = run;
        run += t;
    }
}

__global__ __launch_bounds__(kBlk) void k_home_order(DevBox B, const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ bsum, int32_t* home, int64_t n) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < B.ncells;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = (int64_t)off[c] + bsum[c / kScanCells];
        const int32_t cnt = B.count[c] < B.cap ? B.count[c] : B.cap;
        for (int32_t k = 0; k < cnt && o + k < n; ++k) home[o + k] = (int32_t)(c * B.cap + k);
    }
}

// ------------------------------------------------------ cell-list total
constexpr int kUnroll = 4;   // candidate records requested together

// Does the stencil of cell (cx, cy, cz) stay clear of the periodic wrap with room
// to spare?  Then every candidate lies within (k + 1) S < L/2 of the home
// particle along each axis (at least 2k + 3 cells per axis: half a cell of
// margin, far above the rounding of the cell assignment), and the minimum
// image of a coordinate difference is the difference itself, bit for bit.
__device__ __forceinline__ bool stencil_inside(const DevBox& B, int32_t cx, int32_t cy, int32_t cz) {
    const int32_t c[3] = {cx, cy, cz};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        in = in && B.M[a] >= 2 * B.k[a] + 3 && c[a] >= B.k[a] && c[a] <= B.M[a] - 1 - B.k[a];
    return in;
}

__device__ __forceinline__ double image_diff(double d, double L, double hL, bool wrap) {
    return wrap ? nearest_image(d, L, hL) : d;
}

// e_i of one home particle over its stencil (WRAP: apply the minimum image).
// In-cutoff pairs wait in a per-wavefront ring in LDS until 64 are queued; then
// every lane takes one and evaluates the Lennard-Jones term (about one
// candidate in six lies inside the cutoff of a full stencil, so the pair
// arithmetic runs at full lane occupancy instead of under a mostly empty mask)
// and adds it to its home particle's accumulator with an LDS atomic.
constexpr int kRing = 128;   // queued pairs per wavefront (at most 63 + 64 at a time)

struct PairQueue {
    double* r2;      // [kRing] squared distances
    int32_t* meta;   // [kRing] home lane | species pair << 8
    double* acc;     // [kWave] energy of each lane's home particle
};

template <bool MIX, bool VIR>
__device__ __forceinline__ void drain_pairs(const PassConst& K, const double* te4, const double* ts2,
                                            const PairQueue& Q, uint32_t head, uint32_t cnt, int lane) {
    // the ring entries written by other lanes of this wavefront are visible to every lane
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    if ((uint32_t)lane < cnt) {
        const uint32_t e = (head + (uint32_t)lane) & (kRing - 1);
        const double r2 = Q.r2[e];
        const int32_t mt = Q.meta[e];
        const int q = mt >> 8;
        const double e4 = MIX ? te4[q] : K.e4, s2 = MIX ? ts2[q] : K.s2;
        const double v = VIR ? lj_virial_from_r2(r2, K.rc2, e4, s2) : lj_from_r2(r2, K.rc2, e4, s2);
        atomicAdd(&Q.acc[mt & (kWave - 1)], v);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
}

// Energy (or pair virial) of each lane's home particle over its stencil.  Every
// lane of the wavefront calls it (lanes without a home particle pass live =
// false and have no candidates); the loops run to the wavefront's largest cell
// count so that the queue is drained with all lanes active.  HALF: each pair
// once, for a total only -- the stencil offsets after (0, 0, 0) in z, y, x
// order and, in the home cell, the particles with a larger id (the stencil is
// symmetric and no axis is covered whole, so every other pair of cells is
// reached from exactly one side).
template <bool MIX, bool VIR, bool WRAP, bool HALF>
__device__ __forceinline__ double home_energy(const DevBox& B, const PassConst& K, const uint32_t* tab,
                                              const double* te4, const double* ts2, const double4& me, int32_t myid,
                                              int sa, int ns, int32_t cx, int32_t cy, int32_t cz, bool live,
                                              const PairQueue& Q) {
    const int lane = threadIdx.x & (kWave - 1);
    Q.acc[lane] = 0.0;
    uint32_t head = 0, tail = 0;   // wave-uniform positions in the ring
    for (int t = 0; t < B.nstencil; ++t) {
        const uint32_t pk = tab[t];
        bool centre = false;
        if (HALF) {
            const int32_t ox = (int32_t)(pk & 0x3FF) - B.k[0], oy = (int32_t)((pk >> 10) & 0x3FF) - B.k[1];
            const int32_t oz = (int32_t)(pk >> 20) - B.k[2];
            if (oz < 0 || (oz == 0 && (oy < 0 || (oy == 0 && ox < 0)))) continue;
            centre = (ox | oy | oz) == 0;
        }
        const int64_t nb = stencil_cell(B, pk, cx, cy, cz);
        const int32_t nc = live ? gload(B.count + nb) : 0;
        const int32_t ncmax = wave_max_i32_uniform(nc);
        const double4* ne = B.ent + nb * B.cap;
        for (int j = 0; j < ncmax; j += kUnroll) {
            double4 o[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) o[u] = gload(ne + (j + u < nc ? j + u : 0));
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                bool in = false;
                double r2 = 0.0;
                int q = 0;
                const int32_t oid = meta_low(o[u].w);
                if (j + u < nc && (HALF && centre ? oid > myid : oid != myid)) {
                    const double dx = image_diff(o[u].x - me.x, K.L[0], K.hL[0], WRAP);
                    const double dy = image_diff(o[u].y - me.y, K.L[1], K.hL[1], WRAP);
                    const double dz = image_diff(o[u].z - me.z, K.L[2], K.hL[2], WRAP);
                    r2 = (dx * dx + dy * dy) + dz * dz;
                    q = MIX ? sa * ns + meta_species(o[u].w) : 0;
                    // (a pair with eps = 0 is queued too and adds zero)
                    in = r2 < K.rc2;
                }
                const uint64_t m = __ballot(in);
                if (in) {
                    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    const uint32_t e = (tail + below) & (kRing - 1);
                    Q.r2[e] = r2;
                    Q.meta[e] = lane | (q << 8);
                }
                tail += (uint32_t)__builtin_popcountll(m);
                if (tail - head >= (uint32_t)kWave) {
                    drain_pairs<MIX, VIR>(K, te4, ts2, Q, head, kWave, lane);
                    head += kWave;
                }
            }
        }
    }
    if (tail != head) drain_pairs<MIX, VIR>(K, te4, ts2, Q, head, tail - head, lane);
    return Q.acc[lane];
}

// Per-particle energies e_i; partial[blockIdx] = sum of e_i of the block.
// VIR: the pair virial -r du/dr in place of the pair energy (pressure).
// HALF: each pair once (no e_out); the partial is twice the block's sum of
// pairs, exactly, so that the finish's half of the sum is the sum of pairs.
template <bool MIX, bool VIR = false, bool HALF = false>
__global__ __launch_bounds__(kBlk) void k_total_cells(const DevBox* __restrict__ boxp, const int32_t* __restrict__ home,
                                                       int64_t n, double* e_out, double* partial) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ double red[kBlk / kWave];
    __shared__ double te4[kMaxSpecies * kMaxSpecies], ts2[kMaxSpecies * kMaxSpecies];
    __shared__ double q_r2[kBlk / kWave][kRing];
    __shared__ int32_t q_meta[kBlk / kWave][kRing];
    __shared__ double q_acc[kBlk];
    const DevBox& B = *boxp;
    load_stencil(B, tab);
    load_species_tables(B, te4, ts2);
    const PassConst K = pass_const(B);
    __syncthreads();
    const int w = threadIdx.x / kWave;
    const PairQueue Q{q_r2[w], q_meta[w], q_acc + w * kWave};
    const int64_t h = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const bool live = h < n;
    int32_t slot = live ? home[h] : 0;
    if (slot < 0 || (int64_t)slot >= B.ncells * B.cap) slot = 0;   // counters and N disagree: stay in bounds
    const int64_t c = slot / B.cap;
    const double4 me = gload(B.ent + slot);
    const int32_t myid = meta_low(me.w);
    const int sa = meta_species(me.w);
    const int ns = uni(B.ns);
    int32_t cx, cy, cz;
    cell_coords(B, c, cx, cy, cz);
    // the wrap is skipped when no lane of the wavefront needs it
    double ei;
    if (__ballot(live && !stencil_inside(B, cx, cy, cz)) != 0)
        ei = home_energy<MIX, VIR, true, HALF>(B, K, tab, te4, ts2, me, myid, sa, ns, cx, cy, cz, live, Q);
    else
        ei = home_energy<MIX, VIR, false, HALF>(B, K, tab, te4, ts2, me, myid, sa, ns, cx, cy, cz, live, Q);
    if (!live) ei = 0.0;
    if (!HALF && live && e_out) e_out[myid] = ei;
    const double s = block_sum(ei, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = HALF ? 2.0 * s : s;
}

// --------------------------------------------------------- all-pairs total
template <bool MIX>
__global__ __launch_bounds__(kBlk) void k_total_allpairs(const DevBox* __restrict__ boxp, double* e_out,
                                                          double* partial) {
    __shared__ double4 tile[kBlk];
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    const PassConst K = pass_const(B);
    const int ns = uni(B.ns);
    const int64_t n = B.st->n;
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const bool own = i < n;
    const double4 me = gload(B.pos + (own ? i : 0));
    const int sa = meta_species(me.w);
    double ei = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kBlk) {
        const int64_t j = j0 + threadIdx.x;
        __syncthreads();
        tile[threadIdx.x] = gload(B.pos + (j < n ? j : 0));
        __syncthreads();
        const int lim = (n - j0) < kBlk ? (int)(n - j0) : kBlk;
        for (int q = 0; q < lim; ++q) {
            const double4 o = tile[q];
            if (own && j0 + q != i) {
                const double r2 = pass_dist2(K, me.x, me.y, me.z, o.x, o.y, o.z);
                if (MIX) {
                    const int qq = sa * ns + meta_species(o.w);
                    ei += lj_from_r2(r2, K.rc2, B.eps4[qq], B.sig2[qq]);
                } else {
                    ei += lj_from_r2(r2, K.rc2, K.e4, K.s2);
                }
            }
        }
    }
    if (own && e_out) e_out[i] = ei;
    const double s = block_sum(ei, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// U_pair = 0.5 * sum(partial) in a fixed order; U_tail from the species
// counts; the running pair energy is reset to U_pair.
__global__ __launch_bounds__(kBlk) void k_total_finish(const DevBox* __restrict__ boxp, const double* partial,
                                                        int64_t np, double* U) {
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < np; q += kBlk) s += partial[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        const double up = 0.5 * s;
        double ut = 0.0;
        for (int a = 0; a < B.ns; ++a)
            for (int b = 0; b < B.ns; ++b)
                ut += (double)B.st->nsp[a] * (double)B.st->nsp[b] * B.tailK[a * B.ns + b];
        U[0] = up;
        U[1] = ut;
        if (B.st->error == GCMC_OK) B.st->u_pair = up;
    }
}

// The virial W = sum over pairs inside the cutoff of -r du/dr (half the sum of
// the per-particle sums, in a fixed order) and the pressure
// P = N / (beta V) + W / (3V) + P_tail, P_tail the pressure of the full potential
// beyond r_c: (16 pi / (3 V^2)) sum_ab N_a N_b eps_ab sigma_ab^3 [(2/3) q^9 - q^3],
// q = sigma_ab / r_c.
__global__ __launch_bounds__(kBlk) void k_virial_finish(const DevBox* __restrict__ boxp, const double* partial,
                                                         int64_t np, double* out) {
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < np; q += kBlk) s += partial[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        const double W = 0.5 * s;
        const double rc = sqrt(B.rc2);
        double pt = 0.0;
        for (int a = 0; a < B.ns; ++a)
            for (int b = 0; b < B.ns; ++b) {
                const int k = a * B.ns + b;
                const double sig = sqrt(B.sig2[k]);
                const double q3 = (sig / rc) * (sig / rc) * (sig / rc);
                const double eps = 0.25 * B.eps4[k];
                pt += (double)B.st->nsp[a] * (double)B.st->nsp[b] * eps * (sig * sig * sig) *
                      ((2.0 / 3.0) * (q3 * q3 * q3) - q3);
            }
        pt *= 16.0 * M_PI / (3.0 * B.V * B.V);
        out[0] = W;
        out[1] = (double)B.st->n / (B.beta * B.V) + W / (3.0 * B.V) + pt;
        if (B.st->error == GCMC_OK) B.st->w_pair = W;
    }
}

// ------------------------------------------------------ all-pairs moves
// The trial of move m of the all-pairs chain, or of a caller-given move.
struct APTrial {
    int type, npos, sp;
    int64_t idx;
    double p[2][3];
    bool valid;
};

__device__ __forceinline__ void ap_chunk_sums(const DevBox& B, const APTrial& T, int64_t n, int64_t j0,
                                              int64_t j1, bool mix, double& sa, double& sb, double& wa, double& wb) {
    sa = 0.0;
    sb = 0.0;
    wa = 0.0;
    wb = 0.0;
    const PassConst K = pass_const(B);
    const int ns = uni(B.ns);
    for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
        if (j == T.idx) continue;
        const double4 o = gload(B.pos + j);
        int q = 0;
        if (mix) q = T.sp * ns + meta_species(o.w);
        const double e4 = mix ? B.eps4[q] : K.e4, s2 = mix ? B.sig2[q] : K.s2;
        const double r2a = pass_dist2(K, T.p[0][0], T.p[0][1], T.p[0][2], o.x, o.y, o.z);
        sa += lj_uw_from_r2(r2a, K.rc2, e4, s2, wa);
        if (T.npos == 2) {
            const double r2b = pass_dist2(K, T.p[1][0], T.p[1][1], T.p[1][2], o.x, o.y, o.z);
            sb += lj_uw_from_r2(r2b, K.rc2, e4, s2, wb);
        }
    }
}

__device__ __forceinline__ APTrial ap_trial_from_move(const DevBox& B, const gcmc_move& mv, int64_t n) {
    APTrial T;
    T.valid = true;
    T.type = mv.type;
    T.idx = -1;
    T.npos = 1;
    T.sp = 0;
    if (mv.type == GCMC_MOVE_INSERT) {
        T.valid = mv.species >= 0 && mv.species < B.ns;
        T.sp = mv.species;
        T.p[0][0] = mv.x; T.p[0][1] = mv.y; T.p[0][2] = mv.z;
        return T;
    }
    if ((mv.type != GCMC_MOVE_DISPLACE && mv.type != GCMC_MOVE_DELETE) || mv.index < 0 || mv.index >= n) {
        T.valid = false;
        return T;
    }
    T.idx = mv.index;
    const double4 pi = gload(B.pos + T.idx);
    T.sp = meta_species(pi.w);
    T.p[0][0] = pi.x; T.p[0][1] = pi.y; T.p[0][2] = pi.z;
    if (mv.type == GCMC_MOVE_DISPLACE) {
        T.npos = 2;
        T.p[1][0] = mv.x; T.p[1][1] = mv.y; T.p[1][2] = mv.z;
    }
    return T;
}

// grid (chunks, moves): scratch[(m * chunks + chunk) * 4 + {0,1,2,3}] (energy old/new, virial old/new)
__global__ __launch_bounds__(kBlk) void k_delta_ap_partial(const DevBox* __restrict__ boxp, const gcmc_move* moves,
                                                            int64_t chunk, double* scratch) {
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    const int64_t n = B.st->n;
    const int64_t m = blockIdx.y;
    const APTrial T = ap_trial_from_move(B, moves[m], n);
    const int64_t j0 = (int64_t)blockIdx.x * chunk;
    int64_t j1 = j0 + chunk;
    if (j1 > n) j1 = n;
    double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
    if (T.valid) ap_chunk_sums(B, T, n, j0, j1, B.ns > 1, sa, sb, wa, wb);
    sa = block_sum(sa, red);
    sb = block_sum(sb, red);
    wa = block_sum(wa, red);
    wb = block_sum(wb, red);
    if (threadIdx.x == 0) {
        double* o = scratch + (m * gridDim.x + blockIdx.x) * 4;
        o[0] = sa;
        o[1] = sb;
        o[2] = wa;
        o[3] = wb;
    }
}

__global__ __launch_bounds__(kBlk) void k_delta_ap_finish(const DevBox* __restrict__ boxp, const gcmc_move* moves,
                                                           int64_t nchunks, const double* scratch, double* dU_pair,
                                                           double* dU_tail, double* dW_pair) {
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    const int64_t n = B.st->n;
    const int64_t m = blockIdx.x;
    const APTrial T = ap_trial_from_move(B, moves[m], n);
    double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
    for (int64_t q = threadIdx.x; q < nchunks; q += kBlk) {
        const double* o = scratch + (m * nchunks + q) * 4;
        sa += o[0];
        sb += o[1];
        wa += o[2];
        wb += o[3];
    }
    sa = block_sum(sa, red);
    sb = block_sum(sb, red);
    wa = block_sum(wa, red);
    wb = block_sum(wb, red);
    if (threadIdx.x == 0) {
        int64_t nsp[kMaxSpecies];
        for (int s = 0; s < kMaxSpecies; ++s) nsp[s] = B.st->nsp[s];
        double p, t, w;
        if (!T.valid) {
            p = __builtin_nan("");
            t = __builtin_nan("");
            w = __builtin_nan("");
        } else if (T.type == GCMC_MOVE_DISPLACE) {
            p = sb - sa;
            t = 0.0;
            w = wb - wa;
        } else if (T.type == GCMC_MOVE_INSERT) {
            p = sa;
            t = tail_change(B, nsp, T.sp, +1);
            w = wa;
        } else {
            p = -sa;
            t = tail_change(B, nsp, T.sp, -1);
            w = -wa;
        }
        dU_pair[m] = p;
        if (dU_tail) dU_tail[m] = t;
        if (dW_pair) dW_pair[m] = w;
    }
}

// ------------------------------------------------ all-pairs chain (A12)
// Device-side chain bookkeeping of the all-pairs path.
struct APChain {
    uint64_t counter;   // next move counter
    uint64_t ctr0;      // first counter of this call
    int64_t att[3], acc[3];
    double sum_n, sum_u, sum_n2, sum_w;
    int64_t moves_done;
    int64_t candidates, pair_evals;
};

__device__ __forceinline__ APTrial ap_trial_from_draws(const DevBox& B, const U8& u, int64_t n) {
    APTrial T;
    T.valid = true;
    T.sp = 0;
    T.type = (u.u[0] < B.p_disp) ? GCMC_MOVE_DISPLACE : ((u.u[1] < 0.5) ? GCMC_MOVE_DELETE : GCMC_MOVE_INSERT);
    T.idx = -1;
    T.npos = 1;
    if (T.type == GCMC_MOVE_INSERT) {
        for (int a = 0; a < 3; ++a) T.p[0][a] = wrap_into_box(B.L[a] * u.u[4 + a], B.L[a]);
        return T;
    }
    if (n == 0) {
        T.valid = false;
        return T;
    }
    const int64_t i = pick_particle(u.u[2], u.u[7], n);
    T.idx = i;
    const double4 pi = gload(B.pos + i);
    T.p[0][0] = pi.x; T.p[0][1] = pi.y; T.p[0][2] = pi.z;
    if (T.type == GCMC_MOVE_DISPLACE) {
        T.npos = 2;
        for (int a = 0; a < 3; ++a)
            T.p[1][a] = wrap_into_box(T.p[0][a] + B.max_disp * (2.0 * u.u[4 + a] - 1.0), B.L[a]);
    }
    return T;
}

__global__ __launch_bounds__(kBlk) void k_ap_chain_eval(const DevBox* __restrict__ boxp, const APChain* ch,
                                                         int64_t chunk, double* scratch) {
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    if (B.st->error != GCMC_OK) return;
    const int64_t n = B.st->n;
    const U8 u = move_uniforms(B.seed, ch->counter, B.box_id);
    const APTrial T = ap_trial_from_draws(B, u, n);
    const int64_t j0 = (int64_t)blockIdx.x * chunk;
    int64_t j1 = j0 + chunk;
    if (j1 > n) j1 = n;
    double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
    if (T.valid) ap_chunk_sums(B, T, n, j0, j1, false, sa, sb, wa, wb);
    sa = block_sum(sa, red);
    sb = block_sum(sb, red);
    wa = block_sum(wa, red);
    wb = block_sum(wb, red);
    if (threadIdx.x == 0) {
        double* o = scratch + blockIdx.x * 4;
        o[0] = sa;
        o[1] = sb;
        o[2] = wa;
        o[3] = wb;
    }
}

__device__ int commit_ap(const DevBox& B, const APTrial& T, const double4& meta_rec, int64_t n, int32_t& maxc);

__global__ __launch_bounds__(kBlk) void k_ap_chain_decide(const DevBox* __restrict__ boxp, APChain* ch,
                                                           int64_t nchunks, const double* scratch, gcmc_log* log) {
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    BoxState* st = B.st;
    if (st->error != GCMC_OK) return;
    const int64_t n = st->n;
    const uint64_t ctr = ch->counter;
    const U8 u = move_uniforms(B.seed, ctr, B.box_id);
    const APTrial T = ap_trial_from_draws(B, u, n);
    double sa = 0.0, sb = 0.0, wa = 0.0, wb = 0.0;
    for (int64_t q = threadIdx.x; q < nchunks; q += kBlk) {
        sa += scratch[q * 4];
        sb += scratch[q * 4 + 1];
        wa += scratch[q * 4 + 2];
        wb += scratch[q * 4 + 3];
    }
    sa = block_sum(sa, red);
    sb = block_sum(sb, red);
    wa = block_sum(wa, red);
    wb = block_sum(wb, red);
    if (threadIdx.x != 0) return;
    const int64_t m = (int64_t)(ctr - ch->ctr0);
    const double tk = B.tailK[0];
    ch->att[T.type] += 1;
    gcmc_log r;
    r.type = T.type;
    r.flags = 0;
    r.accepted = 0;
    r.dU_pair = 0.0;
    r.dU_tail = 0.0;
    r.arg = 0.0;
    r.dW_pair = 0.0;
    r.x = r.y = r.z = 0.0;
    int64_t n_after = n;
    if (!T.valid) {
        r.index = -1;
        r.flags = 1;
    } else {
        double dUp, dUt, dWp;
        if (T.type == GCMC_MOVE_DISPLACE) {
            dUp = sb - sa;
            dUt = 0.0;
            dWp = wb - wa;
        } else if (T.type == GCMC_MOVE_INSERT) {
            dUp = sa;
            dUt = tk * (2.0 * (double)n + 1.0);
            dWp = wa;
        } else {
            dUp = -sa;
            dUt = tk * (1.0 - 2.0 * (double)n);
            dWp = -wa;
        }
        r.dW_pair = dWp;
        const double dU = dUp + dUt;
        const double arg = accept_log_ratio(B, T.type, dU, n);
        const bool ok = metropolis(arg, dU, u.u[3]);
        r.index = (T.type == GCMC_MOVE_INSERT) ? (int32_t)n : (int32_t)T.idx;
        r.dU_pair = dUp;
        r.dU_tail = dUt;
        r.arg = arg;
        const int w = (T.type == GCMC_MOVE_DISPLACE) ? 1 : 0;
        r.x = T.p[w][0]; r.y = T.p[w][1]; r.z = T.p[w][2];
        const int64_t others = (T.idx >= 0) ? n - 1 : n;
        ch->candidates += others;
        ch->pair_evals += others * T.npos;
        if (ok) {
            int32_t mc = st->maxcount;
            const double4 rec = (T.idx >= 0) ? gload(B.pos + T.idx) : make_double4(0, 0, 0, 0);
            const int e = commit_ap(B, T, rec, n, mc);
            if (e != GCMC_OK) {
                ch->att[T.type] -= 1;
                st->error = e;
                st->error_move = (int64_t)ctr;
                return;
            }
            st->maxcount = mc;
            n_after = n + ((T.type == GCMC_MOVE_INSERT) ? 1 : ((T.type == GCMC_MOVE_DELETE) ? -1 : 0));
            st->n = n_after;
            st->nsp[0] = n_after;
            st->u_pair += dUp;
            st->w_pair += dWp;
            ch->acc[T.type] += 1;
            r.accepted = 1;
        }
    }
    if (log) log[m] = r;
    ch->sum_n += (double)n_after;
    ch->sum_n2 += (double)n_after * (double)n_after;
    ch->sum_u += st->u_pair + tk * (double)n_after * (double)n_after;
    ch->sum_w += st->w_pair;
    ch->moves_done = m + 1;
    ch->counter = ctr + 1;
}

__global__ void k_ap_chain_begin(const DevBox* __restrict__ boxp, APChain* ch, uint64_t ctr0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (ctr0 == GCMC_COUNTER_CONTINUE) ctr0 = (uint64_t)boxp->st->counter;
        ch->counter = ctr0;
        ch->ctr0 = ctr0;
        for (int t = 0; t < 3; ++t) ch->att[t] = ch->acc[t] = 0;
        ch->sum_n = ch->sum_u = ch->sum_n2 = ch->sum_w = 0.0;
        ch->moves_done = 0;
        ch->candidates = ch->pair_evals = 0;
    }
}

__global__ void k_ap_chain_end(const DevBox* __restrict__ boxp, const APChain* ch, gcmc_stats* stats) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const DevBox& B = *boxp;
    ChainSums L;
    L.moves = ch->moves_done;
    for (int t = 0; t < 3; ++t) {
        L.att[t] = ch->att[t];
        L.acc[t] = ch->acc[t];
    }
    L.sum_n = ch->sum_n;
    L.sum_n2 = ch->sum_n2;
    L.sum_u = ch->sum_u;
    L.sum_w = ch->sum_w;
    B.st->counter = (int64_t)ch->counter;
    // in_cutoff is not counted on the all-pairs path (-1)
    finish_launch(B, B.st, L, B.st->n, B.st->u_pair, B.st->w_pair, ch->moves_done, ch->candidates, ch->pair_evals,
                  -1, stats);
}

// The all-pairs chain keeps the cell list up to date as well (same commit).
__device__ int commit_ap(const DevBox& B, const APTrial& T, const double4& rec, int64_t n, int32_t& maxc) {
    const int cap = B.cap;
    auto cell_of = [&](const double* p) {
        const int32_t cx = axis_cell(p[0], B.invS[0], B.M[0]);
        const int32_t cy = axis_cell(p[1], B.invS[1], B.M[1]);
        const int32_t cz = axis_cell(p[2], B.invS[2], B.M[2]);
        return ((int64_t)cz * B.M[1] + cy) * B.M[0] + cx;
    };
    auto remove = [&](int64_t c, int64_t loc) {
        const int32_t nc = gload(B.count + c);
        const int64_t last = c * cap + nc - 1;
        if (loc != last) {
            const double4 e = gload(B.ent + last);
            gstore(B.ent + loc, e);
            gstore_w(B.pos + (meta_low(e.w)), pack_meta(meta_species(e.w), (int32_t)loc));
        }
        gstore(B.count + c, nc - 1);
    };
    if (T.type == GCMC_MOVE_DISPLACE) {
        const int64_t c0 = cell_of(T.p[0]), c1 = cell_of(T.p[1]);
        const int64_t loc = meta_low(rec.w);
        if (c0 == c1) {
            gstore(B.ent + loc, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], pack_meta(T.sp, (int32_t)T.idx)));
            gstore(B.pos + T.idx, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], rec.w));
            return GCMC_OK;
        }
        const int32_t nc = gload(B.count + c1);
        if (nc >= cap) return GCMC_ERR_CELL_OVERFLOW;
        remove(c0, loc);
        const int64_t nl = c1 * cap + nc;
        gstore(B.ent + nl, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], pack_meta(T.sp, (int32_t)T.idx)));
        gstore(B.count + c1, nc + 1);
        gstore(B.pos + T.idx, make_double4(T.p[1][0], T.p[1][1], T.p[1][2], pack_meta(T.sp, (int32_t)nl)));
        if (nc + 1 > maxc) maxc = nc + 1;
        return GCMC_OK;
    }
    if (T.type == GCMC_MOVE_INSERT) {
        if (n >= B.max_n) return GCMC_ERR_CAPACITY;
        const int64_t c0 = cell_of(T.p[0]);
        const int32_t nc = gload(B.count + c0);
        if (nc >= cap) return GCMC_ERR_CELL_OVERFLOW;
        const int64_t nl = c0 * cap + nc;
        gstore(B.ent + nl, make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(T.sp, (int32_t)n)));
        gstore(B.count + c0, nc + 1);
        gstore(B.pos + n, make_double4(T.p[0][0], T.p[0][1], T.p[0][2], pack_meta(T.sp, (int32_t)nl)));
        if (nc + 1 > maxc) maxc = nc + 1;
        return GCMC_OK;
    }
    const int64_t c0 = cell_of(T.p[0]);
    remove(c0, meta_low(rec.w));
    if (T.idx != n - 1) {
        const double4 last = gload(B.pos + (n - 1));
        gstore(B.pos + T.idx, last);
        gstore_w(B.ent + (meta_low(last.w)), pack_meta(meta_species(last.w), (int32_t)T.idx));
    }
    return GCMC_OK;
}

// ------------------------------------------------------------- gradient
// Per particle: dU/dr_i = sum_j (24 eps / r^2)(2 s12 - s6) d_ij, written by
// particle id; parameter partials per block: [0, ns^2) d eps, [ns^2, 2 ns^2)
// d sigma, each pair met twice contributing half from each end.  One lane per
// particle in cell order, as the total energy.

// Force and parameter-derivative sums of each lane's home particle over its
// stencil (WRAP: apply the minimum image), organised like the energy pass:
// the candidate loop only forms the distance vector and r^2, the pairs inside
// the cutoff wait in a per-wavefront ring in LDS, and every 64 of them are
// evaluated one per lane (the force coefficient and the two parameter terms)
// and added to their home particle's sums with LDS atomics, so the pair
// arithmetic runs at full lane occupancy instead of under a mostly empty mask.
// teo[q] = eps4 / sigma of species pair q (the sigma derivative's prefactor, so
// no pair takes a square root).
struct GradQueue {
    double* dx;   // [kRing] each: the distance vector (r^2 is formed again from it, bit for bit)
    double* dy;
    double* dz;
    int32_t* meta;   // [kRing] home lane | other species << 8 | species pair << 16
    double* gx;      // [kWave] force sums of each lane's home particle
    double* gy;
    double* gz;
    double* de;      // [kWave * S] eps and sigma terms by the other particle's species
    double* ds;
};

// S: a bound on the number of species (1, 2 or kMaxSpecies), the width of the
// per-particle parameter sums in LDS.
template <int S>
__device__ __forceinline__ void drain_grad(const PassConst& K, const double* te4, const double* ts2,
                                           const double* teo, const GradQueue& Q, uint32_t head, uint32_t cnt,
                                           int lane) {
    // the ring entries written by other lanes of this wavefront are visible to every lane
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    if ((uint32_t)lane < cnt) {
        constexpr bool MIX = S > 1;
        const uint32_t e = (head + (uint32_t)lane) & (kRing - 1);
        const double dx = Q.dx[e], dy = Q.dy[e], dz = Q.dz[e];
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const int32_t mt = Q.meta[e];
        const int h = mt & (kWave - 1), sb = (mt >> 8) & 0xFF, q = mt >> 16;
        const double eps4 = MIX ? te4[q] : K.e4, sig2 = MIX ? ts2[q] : K.s2;
        const double ir2 = 1.0 / r2;
        const double sr2 = sig2 * ir2;
        const double s6 = sr2 * sr2 * sr2;
        const double s12 = s6 * s6;
        const double coef = (6.0 * eps4 * ir2) * (2.0 * s12 - s6);
        atomicAdd(&Q.gx[h], coef * dx);
        atomicAdd(&Q.gy[h], coef * dy);
        atomicAdd(&Q.gz[h], coef * dz);
        const int slot = h * S + sb;
        atomicAdd(&Q.de[slot], 0.5 * 4.0 * (s12 - s6));
        atomicAdd(&Q.ds[slot], 0.5 * teo[q] * (12.0 * s12 - 6.0 * s6));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
}

template <int S, bool WRAP>
__device__ __forceinline__ void home_gradient(const DevBox& B, const PassConst& K, const uint32_t* tab,
                                              const double* te4, const double* ts2, const double* teo,
                                              const double4& me, int32_t myid, int sa, int ns, int32_t cx, int32_t cy,
                                              int32_t cz, bool live, const GradQueue& Q) {
    constexpr bool MIX = S > 1;
    const int lane = threadIdx.x & (kWave - 1);
    Q.gx[lane] = Q.gy[lane] = Q.gz[lane] = 0.0;
#pragma unroll
    for (int b = 0; b < S; ++b) {
        Q.de[lane * S + b] = 0.0;
        Q.ds[lane * S + b] = 0.0;
    }
    uint32_t head = 0, tail = 0;   // wave-uniform positions in the ring
    for (int t = 0; t < B.nstencil; ++t) {
        const int64_t nb = stencil_cell(B, tab[t], cx, cy, cz);
        const int32_t nc = live ? gload(B.count + nb) : 0;
        const int32_t ncmax = wave_max_i32_uniform(nc);
        const double4* ne = B.ent + nb * B.cap;
        for (int j = 0; j < ncmax; j += kUnroll) {
            double4 ob[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) ob[u] = gload(ne + (j + u < nc ? j + u : 0));
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const double4& o = ob[u];
                bool in = false;
                double dx = 0.0, dy = 0.0, dz = 0.0;
                int32_t mt = 0;
                if (j + u < nc && meta_low(o.w) != myid) {
                    dx = image_diff(o.x - me.x, K.L[0], K.hL[0], WRAP);
                    dy = image_diff(o.y - me.y, K.L[1], K.hL[1], WRAP);
                    dz = image_diff(o.z - me.z, K.L[2], K.hL[2], WRAP);
                    const double r2 = (dx * dx + dy * dy) + dz * dz;
                    const int sb = MIX ? meta_species(o.w) : 0;
                    mt = lane | (sb << 8) | ((MIX ? sa * ns + sb : 0) << 16);
                    in = r2 < K.rc2 && r2 != 0.0;
                }
                const uint64_t m = __ballot(in);
                if (in) {
                    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    const uint32_t e = (tail + below) & (kRing - 1);
                    Q.dx[e] = dx;
                    Q.dy[e] = dy;
                    Q.dz[e] = dz;
                    Q.meta[e] = mt;
                }
                tail += (uint32_t)__builtin_popcountll(m);
                if (tail - head >= (uint32_t)kWave) {
                    drain_grad<S>(K, te4, ts2, teo, Q, head, kWave, lane);
                    head += kWave;
                }
            }
        }
    }
    if (tail != head) drain_grad<S>(K, te4, ts2, teo, Q, head, tail - head, lane);
    // (drain_grad ends with a wavefront fence: every lane's sums are complete and visible)
}

template <int S>
__global__ __launch_bounds__(kBlk) void k_grad_cells(const DevBox* __restrict__ boxp, const int32_t* __restrict__ home,
                                                      int64_t n, double* grad, double* partial) {
    __shared__ uint32_t tab[kMaxStencil];
    __shared__ double red[kBlk / kWave];
    __shared__ double te4[kMaxSpecies * kMaxSpecies], ts2[kMaxSpecies * kMaxSpecies];
    __shared__ double teo[kMaxSpecies * kMaxSpecies];
    __shared__ double q_dx[kBlk / kWave][kRing], q_dy[kBlk / kWave][kRing], q_dz[kBlk / kWave][kRing];
    __shared__ int32_t q_meta[kBlk / kWave][kRing];
    __shared__ double a_gx[kBlk], a_gy[kBlk], a_gz[kBlk], a_de[kBlk * S], a_ds[kBlk * S];
    const DevBox& B = *boxp;
    load_stencil(B, tab);
    load_species_tables(B, te4, ts2);
    if (threadIdx.x < kMaxSpecies * kMaxSpecies) teo[threadIdx.x] = B.eps4[threadIdx.x] / sqrt(B.sig2[threadIdx.x]);
    const PassConst K = pass_const(B);
    __syncthreads();
    const int w = threadIdx.x / kWave;
    const GradQueue Q{q_dx[w], q_dy[w], q_dz[w], q_meta[w], a_gx + w * kWave, a_gy + w * kWave,
                      a_gz + w * kWave, a_de + w * kWave * S, a_ds + w * kWave * S};
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t h = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const int ns = uni(B.ns);
    const bool own = h < n;
    int32_t slot = own ? home[h] : 0;
    if (slot < 0 || (int64_t)slot >= B.ncells * B.cap) slot = 0;   // counters and N disagree: stay in bounds
    const int64_t c = slot / B.cap;
    const double4 me = gload(B.ent + slot);
    const int32_t myid = meta_low(me.w);
    const int sa = own ? meta_species(me.w) : 0;
    int32_t cx, cy, cz;
    cell_coords(B, c, cx, cy, cz);
    // the wrap is skipped when no lane of the wavefront needs it
    if (__ballot(own && !stencil_inside(B, cx, cy, cz)) != 0)
        home_gradient<S, true>(B, K, tab, te4, ts2, teo, me, myid, sa, ns, cx, cy, cz, own, Q);
    else
        home_gradient<S, false>(B, K, tab, te4, ts2, teo, me, myid, sa, ns, cx, cy, cz, own, Q);
    if (own && grad) {
        grad[myid] = Q.gx[lane];
        grad[n + myid] = Q.gy[lane];
        grad[2 * n + myid] = Q.gz[lane];
    }
    // parameter partials: entry (a, b) gets the lanes with own species a
    for (int a = 0; a < ns; ++a) {
        for (int b = 0; b < ns; ++b) {
            const bool mine = own && sa == a;
            const int k = lane * S + b;
            const double ve = block_sum(mine ? Q.de[k] : 0.0, red);
            const double vs = block_sum(mine ? Q.ds[k] : 0.0, red);
            if (threadIdx.x == 0) {
                partial[(size_t)blockIdx.x * 2 * kMaxSpecies * kMaxSpecies + a * ns + b] = ve;
                partial[(size_t)blockIdx.x * 2 * kMaxSpecies * kMaxSpecies + kMaxSpecies * kMaxSpecies + a * ns + b] =
                    vs;
            }
        }
    }
}

// Sum the parameter partials in order and add the tail-correction terms.
__global__ __launch_bounds__(kBlk) void k_grad_finish(const DevBox* __restrict__ boxp, const double* partial,
                                                       int64_t np, double* deps, double* dsig) {
    __shared__ double red[kBlk / kWave];
    const DevBox& B = *boxp;
    const int ns = B.ns;
    const int stride = 2 * kMaxSpecies * kMaxSpecies;
    for (int q = 0; q < ns * ns; ++q) {
        double se = 0.0, ss = 0.0;
        for (int64_t b = threadIdx.x; b < np; b += kBlk) {
            se += partial[b * stride + q];
            ss += partial[b * stride + kMaxSpecies * kMaxSpecies + q];
        }
        se = block_sum(se, red);
        ss = block_sum(ss, red);
        if (threadIdx.x == 0) {
            const int a = q / ns, b = q % ns;
            const double pre = (8.0 * M_PI / (3.0 * B.V)) * (double)B.st->nsp[a] * (double)B.st->nsp[b];
            const double e = 0.25 * B.eps4[q], s = sqrt(B.sig2[q]);
            const double x = s / sqrt(B.rc2), x3 = x * x * x, x9 = x3 * x3 * x3;
            if (deps) deps[q] = se + pre * (s * s * s) * (x9 / 3.0 - x3);
            if (dsig) dsig[q] = ss + pre * e * (s * s) * (4.0 * x9 - 6.0 * x3);
        }
    }
}

// ------------------------------------------------------------ launchers
// Scratch layout of a cell-list pass (in doubles): the block partials (times
// `stride` doubles per block), then, as int32, the particles in cell order
// (n), the cell offsets (ncells) and the scan-block totals.
// Each pair once needs a stencil that reaches every other pair of cells from
// exactly one side: no axis it covers whole.
static bool half_stencil_ok(const DevBox& hb) { return !(hb.full[0] | hb.full[1] | hb.full[2]); }
static int64_t cell_pass_blocks(int64_t n) { return n > 0 ? (n + kBlk - 1) / kBlk : 1; }
static int64_t scan_blocks(const DevBox& hb) { return (hb.ncells + kScanCells - 1) / kScanCells; }
static int64_t cell_pass_doubles(const DevBox& hb, int64_t n, int64_t stride) {
    const int64_t ints = n + hb.ncells + scan_blocks(hb);
    return cell_pass_blocks(n) * stride + (ints + 1) / 2 + 1;
}

// The particles in cell order into the scratch after `partial_doubles`.
static int32_t* cell_order(const DevBox& hb, int64_t n, double* scratch, int64_t partial_doubles, hipStream_t s) {
    int32_t* home = reinterpret_cast<int32_t*>(scratch + partial_doubles);
    int32_t* off = home + n;
    int32_t* bsum = off + hb.ncells;
    const int64_t nsb = scan_blocks(hb);
    hipLaunchKernelGGL(k_scan_cells, dim3((unsigned)nsb), dim3(kBlk), 0, s, hb.count, hb.ncells, off, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlk), 0, s, bsum, nsb);
    const int64_t g = (hb.ncells + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(k_home_order, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(kBlk), 0, s, hb, off, bsum, home, n);
    return home;
}

int launch_total(const DevBox& hb, const DevBox* d_box, int32_t maxc, bool all_pairs, double* e_out,
                 double* partial, int64_t partial_len, double* U, hipStream_t s, int64_t n) {
    (void)maxc;
    const bool mix = hb.ns > 1;
    int64_t nb;
    if (all_pairs) {
        nb = (n + kBlk - 1) / kBlk;
        if (nb < 1) nb = 1;
        if (nb > partial_len) return -1;
        if (mix)
            hipLaunchKernelGGL(k_total_allpairs<true>, dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, e_out, partial);
        else
            hipLaunchKernelGGL(k_total_allpairs<false>, dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, e_out, partial);
    } else {
        nb = cell_pass_blocks(n);
        if (cell_pass_doubles(hb, n, 1) > partial_len) return -1;
        const int32_t* home = cell_order(hb, n, partial, nb, s);
        // a total alone takes each pair once
        if (!e_out && half_stencil_ok(hb)) {
            if (mix)
                hipLaunchKernelGGL((k_total_cells<true, false, true>), dim3((unsigned)nb), dim3(kBlk), 0, s, d_box,
                                   home, n, nullptr, partial);
            else
                hipLaunchKernelGGL((k_total_cells<false, false, true>), dim3((unsigned)nb), dim3(kBlk), 0, s, d_box,
                                   home, n, nullptr, partial);
        } else if (mix) {
            hipLaunchKernelGGL(k_total_cells<true>, dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n, e_out,
                               partial);
        } else {
            hipLaunchKernelGGL(k_total_cells<false>, dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n, e_out,
                               partial);
        }
    }
    hipLaunchKernelGGL(k_total_finish, dim3(1), dim3(kBlk), 0, s, d_box, partial, nb, U);
    return 0;
}

int launch_virial(const DevBox& hb, const DevBox* d_box, int32_t maxc, double* partial, int64_t partial_len,
                  double* out, hipStream_t s, int64_t n) {
    (void)maxc;
    const int64_t nb = cell_pass_blocks(n);
    if (cell_pass_doubles(hb, n, 1) > partial_len) return -1;
    const int32_t* home = cell_order(hb, n, partial, nb, s);
    const bool half = half_stencil_ok(hb);
    if (hb.ns > 1 && half)
        hipLaunchKernelGGL((k_total_cells<true, true, true>), dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n,
                           nullptr, partial);
    else if (hb.ns > 1)
        hipLaunchKernelGGL((k_total_cells<true, true>), dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n,
                           nullptr, partial);
    else if (half)
        hipLaunchKernelGGL((k_total_cells<false, true, true>), dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n,
                           nullptr, partial);
    else
        hipLaunchKernelGGL((k_total_cells<false, true>), dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n,
                           nullptr, partial);
    hipLaunchKernelGGL(k_virial_finish, dim3(1), dim3(kBlk), 0, s, d_box, partial, nb, out);
    return 0;
}

int64_t total_partials_needed(const DevBox& hb, int32_t maxc, bool all_pairs, int64_t n) {
    (void)maxc;
    if (all_pairs) return (n + kBlk - 1) / kBlk + 1;
    return cell_pass_doubles(hb, n, 1);
}

int64_t grad_partials_needed(const DevBox& hb, int32_t maxc, int64_t n) {
    (void)maxc;
    return cell_pass_doubles(hb, n, 2 * kMaxSpecies * kMaxSpecies);
}

int launch_grad(const DevBox& hb, const DevBox* d_box, int32_t maxc, double* grad, double* partial, double* deps,
                double* dsig, hipStream_t s, int64_t n) {
    (void)maxc;
    const int64_t nb = cell_pass_blocks(n);
    const int32_t* home = cell_order(hb, n, partial, nb * 2 * kMaxSpecies * kMaxSpecies, s);
    // the width of the per-particle parameter sums in LDS: 1, 2 or up to kMaxSpecies species
    if (hb.ns > 2)
        hipLaunchKernelGGL(k_grad_cells<kMaxSpecies>, dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n, grad,
                           partial);
    else if (hb.ns == 2)
        hipLaunchKernelGGL(k_grad_cells<2>, dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n, grad, partial);
    else
        hipLaunchKernelGGL(k_grad_cells<1>, dim3((unsigned)nb), dim3(kBlk), 0, s, d_box, home, n, grad, partial);
    if (deps || dsig)
        hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(kBlk), 0, s, d_box, partial, nb, deps, dsig);
    return 0;
}

int64_t ap_chunk_len() { return 8 * kBlk; }

int launch_delta_allpairs(const DevBox* d_box, int64_t n, const gcmc_move* moves, int64_t n_moves, double* scratch,
                          double* dp, double* dt, double* dw, hipStream_t s) {
    const int64_t chunk = ap_chunk_len();
    int64_t nch = (n + chunk - 1) / chunk;
    if (nch < 1) nch = 1;
    if (n_moves > 65535) return -1;
    hipLaunchKernelGGL(k_delta_ap_partial, dim3((unsigned)nch, (unsigned)n_moves), dim3(kBlk), 0, s, d_box, moves,
                       chunk, scratch);
    hipLaunchKernelGGL(k_delta_ap_finish, dim3((unsigned)n_moves), dim3(kBlk), 0, s, d_box, moves, nch, scratch, dp,
                       dt, dw);
    return 0;
}

size_t ap_chain_state_bytes() { return sizeof(APChain); }

void launch_ap_chain_begin(const DevBox* d_box, void* ch, uint64_t ctr0, hipStream_t s) {
    hipLaunchKernelGGL(k_ap_chain_begin, dim3(1), dim3(64), 0, s, d_box, (APChain*)ch, ctr0);
}

void launch_ap_chain_move(const DevBox* d_box, void* ch, int64_t nch, double* scratch, gcmc_log* log,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_ap_chain_eval, dim3((unsigned)nch), dim3(kBlk), 0, s, d_box, (const APChain*)ch,
                       ap_chunk_len(), scratch);
    hipLaunchKernelGGL(k_ap_chain_decide, dim3(1), dim3(kBlk), 0, s, d_box, (APChain*)ch, nch, scratch, log);
}

void launch_ap_chain_end(const DevBox* d_box, const void* ch, gcmc_stats* stats, hipStream_t s) {
    hipLaunchKernelGGL(k_ap_chain_end, dim3(1), dim3(64), 0, s, d_box, (const APChain*)ch, stats);
}

}  // namespace gcmc
