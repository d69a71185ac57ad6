// Internal definitions shared by the gfx950 kernels and the host side of the
// C ABI: the device box descriptor, the device-resident box state and the
// device math (Philox4x32-10, minimum image, Lennard-Jones, wavefront sums).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/gcmc.h"

namespace gcmc {

constexpr int kWave = 64;
constexpr int kMaxSpecies = GCMC_MAX_SPECIES;
constexpr int kMaxStencil = 1024;   // stencil cells kept in LDS

// Sums of the chain statistics over many moves (per launch, or cumulative in
// the box since it was created, imported or cleared).
struct ChainSums {
    int64_t moves;
    int64_t att[3], acc[3];
    double sum_n, sum_n2, sum_u, sum_w;   // N, N^2, u_pair + u_tail and W after each move
};

// Device-resident mutable state of one box.
struct BoxState {
    int64_t n;            // particle count N
    double u_pair;        // running pair energy
    int32_t maxcount;     // upper bound of every cell's count (monotone)
    int32_t error;        // latched GCMC_ERR_*
    int64_t error_move;   // move counter of the error, -1 if none
    int64_t nsp[kMaxSpecies];  // particles per species
    int64_t counter;      // move counter after the last move the chain ran
    double w_pair;        // running pair virial
    ChainSums cum;        // cumulative statistics (part of a checkpoint)
};

// Everything a kernel needs about one box (read-only during a launch).
// Particle record (pos) and cell entry (ent) are both 32 bytes:
//   pos[i] = {x, y, z, meta}, meta = (species << 32) | loc, loc = c * cap + k
//   ent[c * cap + k] = {x, y, z, meta}, meta = (species << 32) | particle id
struct DevBox {
    double4* pos;
    double4* ent;
    int32_t* count;
    BoxState* st;
    double L[3];
    double hL[3];        // 0.5 * L
    double invS[3];      // M / L
    int32_t M[3];
    int32_t span[3];     // stencil cells per axis
    int32_t k[3];        // stencil half-width
    int32_t full[3];     // 1 if the stencil covers the whole axis
    int32_t cap;
    int32_t ns;
    int64_t ncells;
    int64_t max_n;
    double rc2;
    double beta, mu, lambda3, max_disp, p_disp;
    double V;
    double eps4[kMaxSpecies * kMaxSpecies];   // 4 * eps_ab
    double sig2[kMaxSpecies * kMaxSpecies];   // sigma_ab^2
    double tailK[kMaxSpecies * kMaxSpecies];  // (8 pi / 3V) eps sigma^3 (q^9/3 - q^3), q = sigma / rc
    double ptailK[kMaxSpecies * kMaxSpecies]; // (16 pi / 3V^2) eps sigma^3 ((2/3) q^9 - q^3): P_tail / (N_a N_b)
    uint64_t seed;
    uint32_t box_id;
    int32_t nstencil;    // stencil cells kept (at most span_x * span_y * span_z)
    int32_t wait_limit;  // polls of an in-kernel wait before it fails: 0 the default bound, < 0 at once
    const uint32_t* stab;   // the kept stencil slots, packed tx | ty << 10 | tz << 20 (device)
};

// ------------------------------------------------------- uniform values
// readfirstlane of a value every lane holds: the result lives in scalar
// registers and, unlike a field loaded from the descriptor, is not reloaded
// from memory inside loops.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Polls of a bounded in-kernel wait (a flag another wavefront of the workgroup
// sets) before the kernel gives up with GCMC_ERR_INTERNAL.
constexpr int32_t kWaitPollsDefault = 1 << 26;
__host__ __device__ __forceinline__ int32_t wait_bound(int32_t wait_limit) {
    return wait_limit == 0 ? kWaitPollsDefault : wait_limit;
}
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double unid(double v) {
    return __builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, v)));
}
template <class T>
__device__ __forceinline__ T* unip(T* p) {
    return (T*)(uintptr_t)uni64((int64_t)(uintptr_t)p);
}

// Accesses through the box's arrays as global-memory (address space 1)
// operations.  The pointers reach the kernels inside a descriptor, so the
// compiler would otherwise issue flat_* accesses, and a flat access also
// counts against the LDS wait counter: every LDS wait after it would wait for
// the memory operation as well.
typedef double gcmc_d4v __attribute__((ext_vector_type(4)));
#define GCMC_GLOBAL_AS __attribute__((address_space(1)))

__device__ __forceinline__ double4 gload(const double4* p) {
    const gcmc_d4v v = *(const GCMC_GLOBAL_AS gcmc_d4v*)p;
    return make_double4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore(double4* p, const double4& v) {
    const gcmc_d4v w = {v.x, v.y, v.z, v.w};
    *(GCMC_GLOBAL_AS gcmc_d4v*)p = w;
}
__device__ __forceinline__ void gstore_w(double4* p, double w) {   // the fourth component only
    *((GCMC_GLOBAL_AS double*)p + 3) = w;
}
__device__ __forceinline__ int32_t gload(const int32_t* p) { return *(const GCMC_GLOBAL_AS int32_t*)p; }
__device__ __forceinline__ uint32_t gload(const uint32_t* p) { return *(const GCMC_GLOBAL_AS uint32_t*)p; }
__device__ __forceinline__ void gstore(int32_t* p, int32_t v) { *(GCMC_GLOBAL_AS int32_t*)p = v; }

// ------------------------------------------------------------------ packing
__host__ __device__ __forceinline__ double pack_meta(int32_t species, int32_t low) {
    uint64_t v = ((uint64_t)(uint32_t)species << 32) | (uint64_t)(uint32_t)low;
    return __builtin_bit_cast(double, v);
}
__host__ __device__ __forceinline__ int32_t meta_low(double m) {
    return (int32_t)(uint32_t)__builtin_bit_cast(uint64_t, m);
}
__host__ __device__ __forceinline__ int32_t meta_species(double m) {
    return (int32_t)(__builtin_bit_cast(uint64_t, m) >> 32);
}

// -------------------------------------------------------- Philox4x32-10
// Salmon et al., SC'11: ten rounds of two 32x32->64 products with the round
// multipliers, key bumped by the Weyl constants between rounds.
struct U8 { double u[8]; };

__device__ __forceinline__ void philox_block(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double to_unit(uint32_t a, uint32_t b) {
    // 27 + 26 random bits -> a multiple of 2^-53 in [0, 1)
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * 0x1.0p-53;
}

// The eight uniforms of move `ctr` of box `box` (layout documented in gcmc.h).
__device__ __forceinline__ U8 move_uniforms(uint64_t seed, uint64_t ctr, uint32_t box) {
    U8 o;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        uint32_t c0 = (uint32_t)ctr, c1 = (uint32_t)(ctr >> 32), c2 = box, c3 = j;
        philox_block(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
        o.u[2 * j] = to_unit(c0, c1);
        o.u[2 * j + 1] = to_unit(c2, c3);
    }
    return o;
}

// The same eight uniforms with a quarter of the vector work: lane j (mod 4)
// computes Philox block j and the sixteen words are read from lanes 0..3.
// Every lane of the wavefront must be active.
__device__ __forceinline__ double read_lane(double v, int lane);
__device__ __forceinline__ U8 move_uniforms_lanes(uint64_t seed, uint64_t ctr, uint32_t box) {
    uint32_t c0 = (uint32_t)ctr, c1 = (uint32_t)(ctr >> 32), c2 = box, c3 = (uint32_t)(__lane_id() & 3);
    philox_block(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double a = to_unit(c0, c1), b = to_unit(c2, c3);
    U8 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        o.u[2 * j] = read_lane(a, j);
        o.u[2 * j + 1] = read_lane(b, j);
    }
    return o;
}

// ------------------------------------------------------------- geometry
// Minimum image along one axis of length L (h = L/2), coordinates in [0, L):
// d - L if d > h, d + L if d < -h, else d (two selects, no branches; the
// second select cannot fire after the first did, since |d| < L).
__device__ __forceinline__ double nearest_image(double d, double L, double h) {
    const double a = d > h ? d - L : d;
    return a < -h ? a + L : a;
}

__device__ __forceinline__ double wrap_into_box(double x, double L) {
    if (x >= L) x -= L;
    else if (x < 0.0) x += L;
    if (x >= L) x = 0.0;
    return x;
}

// The particle a displacement (Algorithm 2) or a deletion (Algorithm 5)
// picks among n >= 1: uniform over 0 .. n-1.  With 2^b the smallest power of
// two >= n, the 53 random bits of u7 (u7 = k 2^-53) form floor(53 / b) fields
// of b bits, high field first; the pick is the first field below n, else
// min(floor(u2 n), n - 1).  A field below n names the same particle for every
// N above it, so a move evaluated before an earlier insertion or deletion is
// decided almost always keeps its particle.
__device__ __forceinline__ int64_t pick_particle(double u2, double u7, int64_t n) {
    if (n <= 1) return 0;
    const int b = 64 - __clzll((long long)(n - 1));
    const uint64_t k = (uint64_t)(u7 * 9007199254740992.0);
    const uint64_t mask = (1ull << b) - 1ull;
    for (int sh = 53 - b; sh >= 0; sh -= b) {
        const uint64_t v = (k >> sh) & mask;
        if (v < (uint64_t)n) return (int64_t)v;
    }
    const int64_t i = (int64_t)floor(u2 * (double)n);
    return i > n - 1 ? n - 1 : i;
}

__device__ __forceinline__ int32_t axis_cell(double x, double invS, int32_t M) {
    int32_t c = (int32_t)floor(x * invS);
    return c > M - 1 ? M - 1 : (c < 0 ? 0 : c);
}

// Linear cell index of a point (x fastest).
__device__ __forceinline__ int64_t cell_of_point(const DevBox& B, double x, double y, double z) {
    const int32_t cx = axis_cell(x, B.invS[0], B.M[0]);
    const int32_t cy = axis_cell(y, B.invS[1], B.M[1]);
    const int32_t cz = axis_cell(z, B.invS[2], B.M[2]);
    return ((int64_t)cz * B.M[1] + cy) * B.M[0] + cx;
}

// The box's stencil slots into LDS (all threads of the block take part; the
// caller synchronises before use).
__device__ __forceinline__ void load_stencil(const DevBox& B, uint32_t* tab) {
    for (int t = threadIdx.x; t < B.nstencil; t += blockDim.x) tab[t] = gload(B.stab + t);
}

// Linear cell index of a stencil slot t around centre cell (cx, cy, cz).
__device__ __forceinline__ int64_t stencil_cell(const DevBox& B, uint32_t packed, int32_t cx, int32_t cy,
                                                int32_t cz) {
    const int32_t tx = packed & 0x3FF, ty = (packed >> 10) & 0x3FF, tz = packed >> 20;
    int32_t x = B.full[0] ? tx : cx - B.k[0] + tx;
    int32_t y = B.full[1] ? ty : cy - B.k[1] + ty;
    int32_t z = B.full[2] ? tz : cz - B.k[2] + tz;
    x += (x < 0) ? B.M[0] : 0; x -= (x >= B.M[0]) ? B.M[0] : 0;
    y += (y < 0) ? B.M[1] : 0; y -= (y >= B.M[1]) ? B.M[1] : 0;
    z += (z < 0) ? B.M[2] : 0; z -= (z >= B.M[2]) ? B.M[2] : 0;
    return ((int64_t)z * B.M[1] + y) * B.M[0] + x;
}

// ------------------------------------------------------- Lennard-Jones
// u = 4 eps [(sigma/r)^12 - (sigma/r)^6] inside the cutoff, 0 outside;
// +inf at r = 0 (overlap), 0 for eps = 0.
__device__ __forceinline__ double lj_from_r2(double r2, double rc2, double eps4, double sig2) {
    if (!(r2 < rc2) || eps4 == 0.0) return 0.0;
    if (r2 == 0.0) return __builtin_inf();
    const double sr2 = sig2 / r2;
    const double s6 = sr2 * sr2 * sr2;
    return eps4 * (s6 * s6 - s6);
}

// Pair energy u and pair virial w = -r du/dr together (the same s6, the same
// cutoff decision): returns u, adds w to `w`.
__device__ __forceinline__ double lj_uw_from_r2(double r2, double rc2, double eps4, double sig2, double& w) {
    if (!(r2 < rc2) || eps4 == 0.0) return 0.0;
    if (r2 == 0.0) {
        w += __builtin_inf();
        return __builtin_inf();
    }
    const double sr2 = sig2 / r2;
    const double s6 = sr2 * sr2 * sr2;
    const double s12 = s6 * s6;
    w += 6.0 * eps4 * (2.0 * s12 - s6);
    return eps4 * (s12 - s6);
}

// Pair virial -r du/dr of the truncated potential inside the cutoff:
// 24 eps [2 (sigma/r)^12 - (sigma/r)^6] (eps4 = 4 eps).
__device__ __forceinline__ double lj_virial_from_r2(double r2, double rc2, double eps4, double sig2) {
    if (!(r2 < rc2) || eps4 == 0.0) return 0.0;
    if (r2 == 0.0) return __builtin_inf();
    const double sr2 = sig2 / r2;
    const double s6 = sr2 * sr2 * sr2;
    return 6.0 * eps4 * (2.0 * (s6 * s6) - s6);
}

__device__ __forceinline__ double dist2(const DevBox& B, double px, double py, double pz, double qx, double qy,
                                        double qz) {
    const double dx = nearest_image(qx - px, B.L[0], B.hL[0]);
    const double dy = nearest_image(qy - py, B.L[1], B.hL[1]);
    const double dz = nearest_image(qz - pz, B.L[2], B.hL[2]);
    return (dx * dx + dy * dy) + dz * dz;
}

// --------------------------------------------------- wavefront reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Cross-lane move of a double by a DPP pattern (each 32-bit half moved).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the wavefront, returned identically to every lane: DPP exchanges
// within quads (xor 1, xor 2) and rotations by 4 and 8 within each row of 16
// leave every lane of a row with that row's sum; the four row sums are then
// read from lanes 0, 16, 32, 48 and added in a fixed order.
__device__ __forceinline__ double wave_sum_uniform(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x124>(v);   // row_ror:4
    v += dpp_move<0x128>(v);   // row_ror:8
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum over the wavefront kept in vector registers (every lane receives it):
// the same DPP steps within rows of 16, then two cross-row exchanges.  For
// sums that only one lane stores, so they take no scalar registers.
__device__ __forceinline__ double wave_sum_vec(double v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x124>(v);
    v += dpp_move<0x128>(v);
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    return v;
}

// Integer sum and maximum over the wavefront with the same DPP pattern,
// returned identically to every lane (no LDS traffic).
template <int CTRL>
__device__ __forceinline__ int32_t dpp_i32(int32_t v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ int32_t wave_sum_i32_uniform(int32_t v) {
    v += dpp_i32<0xB1>(v);
    v += dpp_i32<0x4E>(v);
    v += dpp_i32<0x124>(v);
    v += dpp_i32<0x128>(v);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

__device__ __forceinline__ int32_t wave_max_i32_uniform(int32_t v) {
    int32_t o = dpp_i32<0xB1>(v);
    v = o > v ? o : v;
    o = dpp_i32<0x4E>(v);
    v = o > v ? o : v;
    o = dpp_i32<0x124>(v);
    v = o > v ? o : v;
    o = dpp_i32<0x128>(v);
    v = o > v ? o : v;
    const int32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const int32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    const int32_t ab = a > b ? a : b, cd = c > d ? c : d;
    return ab > cd ? ab : cd;
}

__device__ __forceinline__ int32_t wave_max_i(int32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        int32_t o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// ---------------------------------------------------------- acceptance
// Log of the acceptance ratio (Eqs. 3-5; insertion with exponent
// beta (mu - dU)), then accept iff arg >= 0 or A < exp(arg); NaN rejects.
__device__ __forceinline__ double accept_log_ratio(const DevBox& B, int type, double dU, int64_t n) {
    if (type == GCMC_MOVE_DISPLACE) return -(B.beta * dU);
    if (type == GCMC_MOVE_INSERT) return log(B.V / (B.lambda3 * (double)(n + 1))) + B.beta * (B.mu - dU);
    return log((B.lambda3 * (double)n) / B.V) - B.beta * (B.mu + dU);
}

__device__ __forceinline__ bool metropolis(double arg, double dU, double A) {
    if (dU != dU) return false;
    if (arg >= 0.0) return true;
    return A < exp(arg);
}

// Tail-correction change for inserting (sign = +1) or deleting (sign = -1) a
// particle of species s given the per-species counts.
__device__ __forceinline__ double tail_change(const DevBox& B, const int64_t* nsp, int s, int sign) {
    double acc = 0.0;
    for (int b = 0; b < B.ns; ++b) acc += (double)nsp[b] * B.tailK[s * B.ns + b];
    return (double)(2 * sign) * acc + B.tailK[s * B.ns + s];
}

// End of a chain launch (one thread, single species): write the launch's
// statistics with the averages of N, U and the pressure over its moves (the
// averages Sec. 3.3.4 computes on the GPU), and fold the sums into the box's
// cumulative statistics.  The caller has already stored N, U, W and the
// counter into the box state.
__device__ __forceinline__ void finish_launch(const DevBox& B, BoxState* st, const ChainSums& L, int64_t N, double U,
                                              double W, int64_t stencils, int64_t cand, int64_t evals,
                                              int64_t incut, gcmc_stats* out) {
    ChainSums& c = st->cum;
    c.moves += L.moves;
    for (int t = 0; t < 3; ++t) {
        c.att[t] += L.att[t];
        c.acc[t] += L.acc[t];
    }
    c.sum_n += L.sum_n;
    c.sum_n2 += L.sum_n2;
    c.sum_u += L.sum_u;
    c.sum_w += L.sum_w;
    if (!out) return;
    gcmc_stats o;
    for (int t = 0; t < 3; ++t) {
        o.attempts[t] = L.att[t];
        o.accepts[t] = L.acc[t];
    }
    o.n = N;
    o.moves_done = L.moves;
    o.u_pair = U;
    o.u_tail = B.tailK[0] * (double)N * (double)N;
    o.sum_n = L.sum_n;
    o.sum_u = L.sum_u;
    o.error = st->error;
    o.pad = 0;
    o.error_move = st->error_move;
    o.stencils = stencils;
    o.candidates = cand;
    o.pair_evals = evals;
    o.in_cutoff = incut;
    o.w_pair = W;
    o.sum_w = L.sum_w;
    o.sum_n2 = L.sum_n2;
    const double inv = L.moves > 0 ? 1.0 / (double)L.moves : __builtin_nan("");
    o.avg_n = L.sum_n * inv;
    o.avg_u = L.sum_u * inv;
    o.avg_p = o.avg_n / (B.beta * B.V) + (L.sum_w * inv) / (3.0 * B.V) + B.ptailK[0] * (L.sum_n2 * inv);
    *out = o;
}

}  // namespace gcmc

// ------------------------------------------------------------ host side
struct gcmc_box {
    gcmc::DevBox d;          // host copy of the descriptor
    gcmc::DevBox* d_desc;    // device copy (batched kernels)
    double* scratch;         // reduction partials (library-owned)
    int64_t scratch_len;     // doubles
    void* ap_chain;          // all-pairs chain bookkeeping (device)
    int device;
    int waves, rows;         // launch shape of the move kernels
    int32_t req_m[3];        // cells per axis asked for at create (0 = the paper's rule)
    double h_eps[gcmc::kMaxSpecies * gcmc::kMaxSpecies];   // force-field tables as given (host)
    double h_sig[gcmc::kMaxSpecies * gcmc::kMaxSpecies];
};

constexpr int kMaxBatchGroups = 8;   // launch shapes one batch may mix

struct gcmc_batch {
    gcmc_box** boxes;        // host array, in the caller's order
    int32_t n;
    gcmc::DevBox* d_descs;   // device array, launch order (by group, decreasing N within a group)
    gcmc::DevBox* h_descs;   // what d_descs holds (to detect a rebuilt box)
    int32_t* d_order;        // launch slot -> caller index (device)
    int32_t* h_order;        // the same on the host
    int32_t* by_n;           // caller indices by decreasing N at create
    int32_t ngroups;         // boxes grouped by launch path and shape
    int32_t gstart[kMaxBatchGroups], gcount[kMaxBatchGroups];
    int32_t gkey[kMaxBatchGroups][3];   // path (0 speculative, 1 pipelined, 2 per-move, 3 cell per thread,
                                        // 4 held in LDS), waves, rows
    hipStream_t side[kMaxBatchGroups];  // streams of groups 1.. (created when first needed)
    hipEvent_t ev_fork, ev_join[kMaxBatchGroups];
};

namespace gcmc {
int set_error(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// moves.hip
int launch_chain(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int rows, int64_t n_moves,
                 uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s);
bool chain_cfg_exists(int waves, int rows);

// resident.hip
bool resident_cfg_exists(int waves);
int launch_chain_resident(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                          uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s);

// micro.hip
bool paper_cfg_exists(int waves);
int launch_chain_paper(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                       uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s);

// spec.hip
bool spec_supported(const DevBox& hb);
bool spec_cfg_exists(int waves);
bool async_supported(const DevBox& hb);
bool async_cfg_exists(int waves);
int launch_chain_async(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                       uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s);
int launch_chain_spec(const DevBox* d_boxes, const int32_t* d_order, int n_boxes, int waves, int64_t n_moves,
                      uint64_t ctr0, gcmc_stats* stats, gcmc_log* log, hipStream_t s, int ng);
int spec_needs_groups(const DevBox& hb);
int launch_delta(const DevBox* d_box, bool mix, int64_t n_moves, const gcmc_move* moves, double* dp, double* dt,
                 double* dw, hipStream_t s);
void launch_commit(const DevBox* d_box, const gcmc_move* move, const double* dU, const double* dW, hipStream_t s);
void launch_neighbors(const DevBox* d_box, const double* pts, const int32_t* excl, int64_t n, int32_t max_ids,
                      int32_t* ids, int32_t* counts, hipStream_t s);

// energy.hip
int launch_total(const DevBox& hb, const DevBox* d_box, int32_t maxc, bool all_pairs, double* e_out,
                 double* partial, int64_t partial_len, double* U, hipStream_t s, int64_t n);
int64_t total_partials_needed(const DevBox& hb, int32_t maxc, bool all_pairs, int64_t n);
int launch_virial(const DevBox& hb, const DevBox* d_box, int32_t maxc, double* partial, int64_t partial_len,
                  double* out, hipStream_t s, int64_t n);
int64_t grad_partials_needed(const DevBox& hb, int32_t maxc, int64_t n);
int launch_grad(const DevBox& hb, const DevBox* d_box, int32_t maxc, double* grad, double* partial, double* deps,
                double* dsig, hipStream_t s, int64_t n);
int64_t ap_chunk_len();
int launch_delta_allpairs(const DevBox* d_box, int64_t n, const gcmc_move* moves, int64_t n_moves, double* scratch,
                          double* dp, double* dt, double* dw, hipStream_t s);
size_t ap_chain_state_bytes();
void launch_ap_chain_begin(const DevBox* d_box, void* ch, uint64_t ctr0, hipStream_t s);
void launch_ap_chain_move(const DevBox* d_box, void* ch, int64_t nch, double* scratch, gcmc_log* log,
                          hipStream_t s);
void launch_ap_chain_end(const DevBox* d_box, const void* ch, gcmc_stats* stats, hipStream_t s);

// box.hip
int read_box_state(gcmc_box* box, BoxState* h, hipStream_t s);
int ensure_scratch(gcmc_box* box, int64_t len);
}  // namespace gcmc

#define GCMC_HIP(call)                                                       \
    do {                                                                     \
        hipError_t _e = (call);                                              \
        if (_e != hipSuccess) return gcmc::check_hip(_e, #call);             \
    } while (0)
