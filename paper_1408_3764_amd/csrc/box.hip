// Box lifetime, cell-list construction (binning), inspection and checkpoints.
//
// Binning follows Sec. 3.2.1 of the paper: every particle claims a unique slot
// of its cell with an atomic increment of the cell's counter.  Slot order from
// atomics is arbitrary, so a second pass orders each cell's entries by particle
// index; the layout (and with it every floating-point sum order) is then a
// function of the configuration alone.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "gcmc_internal.h"

namespace gcmc {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int check_hip(hipError_t e, const char* what) {
    return set_error(GCMC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------ kernels
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Copy SoA input into the particle records; flags coordinates outside [0, L)
// and bad species in st->error.
__global__ void k_upload(DevBox B, const double* __restrict__ x, const double* __restrict__ y,
                         const double* __restrict__ z, const int32_t* __restrict__ sp, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double px = x[i], py = y[i], pz = z[i];
        const int32_t s = sp ? sp[i] : 0;
        const bool ok = (px >= 0.0) && (px < B.L[0]) && (py >= 0.0) && (py < B.L[1]) && (pz >= 0.0) &&
                        (pz < B.L[2]) && s >= 0 && s < B.ns;
        if (!ok) atomicMax(&B.st->error, (int32_t)GCMC_ERR_INVALID_ARG);
        B.pos[i] = make_double4(px, py, pz, pack_meta(s, 0));
    }
}

// The block's species counts (wave-uniform per-wavefront totals) and largest
// occupancy, added to the box state with one atomic each per block: atomics
// of every wavefront on the same few words serialise at the L2 and took most of
// a cell build's time.  Every thread of the block calls it.
template <int BLK>
__device__ __forceinline__ void publish_counts(BoxState* st, int ns, const int64_t* nsp, int32_t maxc) {
    __shared__ int64_t s_nsp[BLK / kWave][kMaxSpecies];
    __shared__ int32_t s_max[BLK / kWave];
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < kMaxSpecies; ++q) s_nsp[w][q] = nsp[q];
        s_max[w] = maxc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t mx = 0;
        for (int v = 0; v < BLK / kWave; ++v) mx = s_max[v] > mx ? s_max[v] : mx;
        for (int q = 0; q < ns; ++q) {
            int64_t t = 0;
            for (int v = 0; v < BLK / kWave; ++v) t += s_nsp[v][q];
            if (t) atomicAdd((unsigned long long*)&st->nsp[q], (unsigned long long)t);
        }
        if (mx > 0) atomicMax(&st->maxcount, mx);
    }
}

constexpr int kCountBlocks = 1024;   // grid of the occupancy and sort passes (grid-stride loops)

// Pass 1: occupancy only (to size the cells); the largest count is kept per
// wavefront and published once per block.
__global__ __launch_bounds__(256) void k_count(DevBox B, int64_t n) {
    int32_t mx = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double4 p = B.pos[i];
        const int64_t c = cell_of_point(B, p.x, p.y, p.z);
        const int32_t k = atomicAdd(&B.count[c], 1);
        mx = k + 1 > mx ? k + 1 : mx;
    }
    mx = wave_max_i32_uniform(mx);
    const int64_t none[kMaxSpecies] = {0, 0, 0, 0};
    publish_counts<256>(B.st, 0, none, mx);
}

// Pass 2: claim a slot and write the cell entry.
__global__ void k_bin(DevBox B, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double4 p = B.pos[i];
        const int64_t c = cell_of_point(B, p.x, p.y, p.z);
        const int32_t k = atomicAdd(&B.count[c], 1);
        if (k < B.cap) {
            B.ent[c * B.cap + k] = make_double4(p.x, p.y, p.z, pack_meta(meta_species(p.w), (int32_t)i));
        } else {
            atomicMax(&B.st->error, (int32_t)GCMC_ERR_CELL_OVERFLOW);
        }
    }
}

// Pass 3 (capacities above 64): order each cell by particle id, set the
// back-pointers, and gather the maximum occupancy and the species counts (kept
// per thread, summed per wavefront, published once per block).
__global__ __launch_bounds__(256) void k_sort_cells(DevBox B) {
    int32_t nsp[kMaxSpecies] = {0, 0, 0, 0};
    int32_t maxc = 0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < B.ncells;
         c += (int64_t)gridDim.x * blockDim.x) {
        int32_t cnt = B.count[c];
        if (cnt > B.cap) cnt = B.cap;
        double4* e = B.ent + c * B.cap;
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
            const int32_t id = meta_low(v.w);
            const int sp = meta_species(v.w);
            B.pos[id].w = pack_meta(sp, (int32_t)(c * B.cap + a));
#pragma unroll
            for (int q = 0; q < kMaxSpecies; ++q) nsp[q] += (sp == q) ? 1 : 0;
        }
        maxc = cnt > maxc ? cnt : maxc;
    }
    int64_t tot[kMaxSpecies];
#pragma unroll
    for (int q = 0; q < kMaxSpecies; ++q) tot[q] = wave_sum_i32_uniform(nsp[q]);
    maxc = wave_max_i32_uniform(maxc);
    publish_counts<256>(B.st, B.ns, tot, maxc);
}

// Pass 3 with one wavefront per cell, for capacities up to 64: lane k holds the
// cell's entry k; the ids are unique, so the entry's slot in id order is the
// number of the cell's entries with a smaller id, and every entry is written
// once, straight to its slot (the layout is the one the per-thread sort above
// produces).  Species counts and the largest occupancy are kept per wavefront
// over its cells and published once per block.
__global__ __launch_bounds__(1024) void k_sort_cells_wave(DevBox B) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int ns = B.ns;
    int64_t nsp[kMaxSpecies] = {0, 0, 0, 0};
    int32_t maxc = 0;
    for (int64_t c = wave0; c < B.ncells; c += nwaves) {
        int32_t cnt = B.count[c];
        cnt = __builtin_amdgcn_readfirstlane(cnt > B.cap ? B.cap : cnt);
        if (cnt == 0) continue;
        double4* e = B.ent + c * B.cap;
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
        int32_t id = INT32_MAX;
        if (lane < cnt) {
            v = e[lane];
            id = meta_low(v.w);
        }
        int32_t rank = 0;
        for (int j = 0; j < cnt; ++j) rank += (__builtin_amdgcn_readlane(id, j) < id) ? 1 : 0;
        // every lane's load has completed (the ranks read all ids) before any store below
        if (lane < cnt) {
            e[rank] = v;
            B.pos[id].w = pack_meta(meta_species(v.w), (int32_t)(c * B.cap + rank));
        }
        const int sp = meta_species(v.w);
#pragma unroll
        for (int q = 0; q < kMaxSpecies; ++q) nsp[q] += __popcll(__ballot(lane < cnt && sp == q));
        maxc = cnt > maxc ? cnt : maxc;
    }
    publish_counts<1024>(B.st, ns, nsp, maxc);
}

// keep: a rebuild keeps the latched error, its move, the move counter and the
// cumulative statistics; otherwise (a new box) all of them start afresh.
__global__ void k_reset_state(BoxState* st, int64_t n, double u_pair, double w_pair, int keep) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->n = n;
        st->u_pair = u_pair;
        st->w_pair = w_pair;
        st->maxcount = 0;
        if (!keep) {
            st->error = GCMC_OK;
            st->error_move = -1;
            st->counter = 0;
            st->cum.moves = 0;
            for (int t = 0; t < 3; ++t) st->cum.att[t] = st->cum.acc[t] = 0;
            st->cum.sum_n = st->cum.sum_n2 = st->cum.sum_u = st->cum.sum_w = 0.0;
        }
        for (int s = 0; s < kMaxSpecies; ++s) st->nsp[s] = 0;
    }
}

// Running energy and virial (a NaN marks a value no longer describing the configuration).
__global__ void k_set_running(BoxState* st, double u_pair, double w_pair) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->u_pair = u_pair;
        st->w_pair = w_pair;
    }
}

// The chain part of a checkpoint: running energy and virial, move counter,
// cumulative statistics.
__global__ void k_apply_checkpoint(BoxState* st, gcmc_checkpoint ck) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->u_pair = ck.u_pair;
        st->w_pair = ck.w_pair;
        st->counter = (int64_t)ck.counter;
        st->cum.moves = ck.moves;
        for (int t = 0; t < 3; ++t) {
            st->cum.att[t] = ck.attempts[t];
            st->cum.acc[t] = ck.accepts[t];
        }
        st->cum.sum_n = ck.sum_n;
        st->cum.sum_n2 = ck.sum_n2;
        st->cum.sum_u = ck.sum_u;
        st->cum.sum_w = ck.sum_w;
    }
}

__global__ void k_clear_averages(BoxState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->cum.moves = 0;
        for (int t = 0; t < 3; ++t) st->cum.att[t] = st->cum.acc[t] = 0;
        st->cum.sum_n = st->cum.sum_n2 = st->cum.sum_u = st->cum.sum_w = 0.0;
    }
}

// Affine rescaling of the particle coordinates, x_a -> x_a * r_a, kept in [0, L_a).
__global__ void k_rescale(DevBox B, int64_t n, double rx, double ry, double rz, double Lx, double Ly, double Lz) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double4 p = B.pos[i];
        p.x = wrap_into_box(p.x * rx, Lx);
        p.y = wrap_into_box(p.y * ry, Ly);
        p.z = wrap_into_box(p.z * rz, Lz);
        B.pos[i] = p;
    }
}

// Clear the latched errors a rebuild resolves (a cell overflow, a wait past its bound).
__global__ void k_clear_rebuild_errors(BoxState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0 &&
        (st->error == GCMC_ERR_CELL_OVERFLOW || st->error == GCMC_ERR_INTERNAL)) {
        st->error = GCMC_OK;
    }
}

__global__ void k_get_particles(DevBox B, double* x, double* y, double* z, int32_t* sp) {
    const int64_t n = B.st->n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double4 p = B.pos[i];
        if (x) x[i] = p.x;
        if (y) y[i] = p.y;
        if (z) z[i] = p.z;
        if (sp) sp[i] = meta_species(p.w);
    }
}

__global__ void k_get_cells(DevBox B, int32_t* cell_of, int32_t* count, int32_t* ids) {
    const int64_t n = B.st->n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (cell_of)
        for (int64_t i = t0; i < n; i += stride) cell_of[i] = (int32_t)(meta_low(B.pos[i].w) / B.cap);
    if (count)
        for (int64_t c = t0; c < B.ncells; c += stride) count[c] = B.count[c];
    if (ids)
        for (int64_t q = t0; q < B.ncells * B.cap; q += stride) ids[q] = meta_low(B.ent[q].w);
}

static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

}  // namespace gcmc

using namespace gcmc;

// ------------------------------------------------------------------ host helpers
static int validate_desc(const gcmc_box_desc* d, int64_t n) {
    if (!d) return set_error(GCMC_ERR_INVALID_ARG, "desc is NULL");
    if (d->n_species < 1 || d->n_species > kMaxSpecies)
        return set_error(GCMC_ERR_INVALID_ARG, "n_species must be 1..4");
    if (!d->eps || !d->sigma) return set_error(GCMC_ERR_INVALID_ARG, "eps/sigma tables are NULL");
    if (!(d->rc > 0.0)) return set_error(GCMC_ERR_INVALID_ARG, "rc must be positive");
    for (int a = 0; a < 3; ++a) {
        if (!(d->L[a] > 0.0)) return set_error(GCMC_ERR_INVALID_ARG, "box edges must be positive");
        if (d->rc > 0.5 * d->L[a]) return set_error(GCMC_ERR_INVALID_ARG, "rc > L/2 breaks the minimum image");
        if (d->cell_m[a] < 0) return set_error(GCMC_ERR_INVALID_ARG, "cell_m must be >= 0");
    }
    if (n < 0 || d->max_n < n || d->max_n < 1 || d->max_n > (int64_t)INT32_MAX)
        return set_error(GCMC_ERR_INVALID_ARG, "need 0 <= n <= max_n < 2^31");
    const int ns = d->n_species;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            if (d->eps[a * ns + b] != d->eps[b * ns + a] || d->sigma[a * ns + b] != d->sigma[b * ns + a])
                return set_error(GCMC_ERR_INVALID_ARG, "eps/sigma tables must be symmetric");
            if (!(d->sigma[a * ns + b] > 0.0) || d->eps[a * ns + b] < 0.0)
                return set_error(GCMC_ERR_INVALID_ARG, "need sigma > 0 and eps >= 0");
        }
    if (!(d->beta > 0.0) || !(d->lambda3 > 0.0) || d->max_disp < 0.0 || d->p_disp < 0.0 || d->p_disp > 1.0)
        return set_error(GCMC_ERR_INVALID_ARG, "need beta > 0, lambda3 > 0, max_disp >= 0, 0 <= p_disp <= 1");
    return GCMC_OK;
}

// Stencil slots kept for this grid.  On an axis the stencil does not cover
// whole, slot coordinate t stands for the cell offset d = t - k; the closest
// points of the centre cell and a cell at offset d along that axis are
// max(0, |d| - 1) cells of side S = L / M apart (0 on a covered axis).  A slot
// whose squared gap summed over the axes exceeds rc^2 by a relative 1e-9 holds
// no partner within the cutoff and is dropped (the margin keeps cells whose gap
// is rc up to rounding of the cell assignment).  Slots stay in x-fastest order.
static void stencil_slots(const DevBox& B, double rc, std::vector<uint32_t>& slots) {
    slots.clear();
    const double lim = (rc * rc) * (1.0 + 1e-9);
    for (int tz = 0; tz < B.span[2]; ++tz)
        for (int ty = 0; ty < B.span[1]; ++ty)
            for (int tx = 0; tx < B.span[0]; ++tx) {
                const int t[3] = {tx, ty, tz};
                double g2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    if (B.full[a]) continue;
                    const int d = std::abs(t[a] - B.k[a]);
                    const double g = d > 1 ? (double)(d - 1) * (B.L[a] / (double)B.M[a]) : 0.0;
                    g2 += g * g;
                }
                if (g2 > lim) continue;
                slots.push_back((uint32_t)tx | ((uint32_t)ty << 10) | ((uint32_t)tz << 20));
            }
}

// Cells per axis (the paper's rule, or the caller's count), the stencil
// half-width and extent, and the kept stencil slots.
static int setup_grid(DevBox& B, const gcmc_box_desc* d, std::vector<uint32_t>& slots) {
    for (int a = 0; a < 3; ++a) {
        int64_t m = (int64_t)floor(d->L[a] / d->rc);
        if (m < 3) m = 3;
        if (d->cell_m[a] > 0) m = d->cell_m[a];
        if (m > 1023) return set_error(GCMC_ERR_INVALID_ARG, "at most 1023 cells per axis");
        B.M[a] = (int32_t)m;
        B.invS[a] = (double)m / d->L[a];
        int32_t kk = (int32_t)ceil(d->rc * B.invS[a]);
        if (kk < 1) kk = 1;
        B.k[a] = kk;
        B.full[a] = (2 * kk + 1 >= B.M[a]) ? 1 : 0;
        B.span[a] = B.full[a] ? B.M[a] : 2 * kk + 1;
        B.L[a] = d->L[a];
        B.hL[a] = 0.5 * d->L[a];
    }
    B.ncells = (int64_t)B.M[0] * B.M[1] * B.M[2];
    // cell slots c * cap + k are 32-bit indices (back-pointers, home slots)
    if (d->cell_cap > 0 && B.ncells * (int64_t)d->cell_cap >= ((int64_t)1 << 31))
        return set_error(GCMC_ERR_INVALID_ARG, "cells x cell_cap must stay below 2^31");
    if ((int64_t)B.span[0] * B.span[1] * B.span[2] > 64 * kMaxStencil)
        return set_error(GCMC_ERR_INVALID_ARG, "stencil larger than 1024 cells: use fewer, larger cells");
    stencil_slots(B, d->rc, slots);
    B.nstencil = (int32_t)slots.size();
    if (B.nstencil > kMaxStencil)
        return set_error(GCMC_ERR_INVALID_ARG, "stencil larger than 1024 cells: use fewer, larger cells");
    return GCMC_OK;
}

static void setup_params(DevBox& B, const gcmc_box_desc* d) {
    const int ns = d->n_species;
    B.ns = ns;
    B.rc2 = d->rc * d->rc;
    B.beta = d->beta;
    B.mu = d->mu;
    B.lambda3 = d->lambda3;
    B.max_disp = d->max_disp;
    B.p_disp = d->p_disp;
    B.V = (d->L[0] * d->L[1]) * d->L[2];
    B.seed = d->seed;
    B.box_id = d->box_id;
    B.max_n = d->max_n;
    const double pre = 8.0 * M_PI / (3.0 * B.V);
    const double ppre = 16.0 * M_PI / (3.0 * B.V * B.V);
    for (int a = 0; a < kMaxSpecies * kMaxSpecies; ++a) {
        B.eps4[a] = 0.0;
        B.sig2[a] = 1.0;
        B.tailK[a] = 0.0;
        B.ptailK[a] = 0.0;
    }
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            const double e = d->eps[a * ns + b], s = d->sigma[a * ns + b];
            B.eps4[a * ns + b] = 4.0 * e;
            B.sig2[a * ns + b] = s * s;
            const double q = s / d->rc, q3 = q * q * q;
            B.tailK[a * ns + b] = pre * e * (s * s * s) * (q3 * q3 * q3 / 3.0 - q3);
            B.ptailK[a * ns + b] = ppre * e * (s * s * s) * ((2.0 / 3.0) * (q3 * q3 * q3) - q3);
        }
}

static int auto_cap(int32_t maxcount) {
    int c = (int)ceil(1.5 * maxcount) + 4;
    c = (c + 3) & ~3;
    return c < 8 ? 8 : c;
}

// Bin the first n particles of B.pos into a fresh cell array.
static int bin_particles(gcmc_box* box, int64_t n, hipStream_t s, bool keep, double u_pair, double w_pair) {
    DevBox& B = box->d;
    k_reset_state<<<1, 1, 0, s>>>(B.st, n, u_pair, w_pair, keep ? 1 : 0);
    k_fill_i32<<<grid_for(B.ncells), 256, 0, s>>>(B.count, B.ncells, 0);
    if (n > 0) k_bin<<<grid_for(n), 256, 0, s>>>(B, n);
    if (B.cap <= kWave) {
        // 16 wavefronts per block, one cell at a time each (a cell's loads are a dependent chain)
        const int64_t blocks = std::min<int64_t>((B.ncells + 15) / 16, kCountBlocks);
        k_sort_cells_wave<<<(unsigned)blocks, 1024, 0, s>>>(B);
    } else {
        k_sort_cells<<<std::min(grid_for(B.ncells), kCountBlocks), 256, 0, s>>>(B);
    }
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

static int alloc_cells(gcmc_box* box, int32_t cap) {
    DevBox& B = box->d;
    if (B.ncells * (int64_t)cap >= ((int64_t)1 << 31))
        return set_error(GCMC_ERR_INVALID_ARG, "cells x cell_cap must stay below 2^31");
    if (B.ent) {
        GCMC_HIP(hipFree(B.ent));
        B.ent = nullptr;
    }
    const size_t bytes = (size_t)B.ncells * (size_t)cap * sizeof(double4);
    if (hipMalloc(&B.ent, bytes) != hipSuccess) {
        B.ent = nullptr;
        return set_error(GCMC_ERR_OOM, "cell array allocation failed");
    }
    B.cap = cap;
    return GCMC_OK;
}

static int sync_desc(gcmc_box* box) {
    GCMC_HIP(hipMemcpy(box->d_desc, &box->d, sizeof(DevBox), hipMemcpyHostToDevice));
    return GCMC_OK;
}

static int read_state(gcmc_box* box, BoxState* h, hipStream_t s) {
    GCMC_HIP(hipMemcpyAsync(h, box->d.st, sizeof(BoxState), hipMemcpyDeviceToHost, s));
    GCMC_HIP(hipStreamSynchronize(s));
    return GCMC_OK;
}

namespace gcmc {
int read_box_state(gcmc_box* box, BoxState* h, hipStream_t s) { return read_state(box, h, s); }

int ensure_scratch(gcmc_box* box, int64_t len) {
    if (box->scratch_len >= len) return GCMC_OK;
    if (box->scratch) {
        GCMC_HIP(hipDeviceSynchronize());
        GCMC_HIP(hipFree(box->scratch));
        box->scratch = nullptr;
        box->scratch_len = 0;
    }
    if (hipMalloc(&box->scratch, (size_t)len * sizeof(double)) != hipSuccess) {
        box->scratch = nullptr;
        return set_error(GCMC_ERR_OOM, "scratch allocation failed");
    }
    box->scratch_len = len;
    return GCMC_OK;
}
}  // namespace gcmc

static void free_box(gcmc_box* box) {
    if (!box) return;
    if (box->d.pos) (void)hipFree(box->d.pos);
    if (box->d.ent) (void)hipFree(box->d.ent);
    if (box->d.count) (void)hipFree(box->d.count);
    if (box->d.st) (void)hipFree(box->d.st);
    if (box->d.stab) (void)hipFree((void*)box->d.stab);
    if (box->d_desc) (void)hipFree(box->d_desc);
    if (box->scratch) (void)hipFree(box->scratch);
    if (box->ap_chain) (void)hipFree(box->ap_chain);
    delete box;
}

extern "C" {

const char* gcmc_last_error(void) { return g_last_error.c_str(); }

const char* gcmc_version(void) { return "gcmc-gfx950 0.1"; }

int gcmc_box_create(const gcmc_box_desc* desc, const double* d_x, const double* d_y, const double* d_z,
                    const int32_t* d_species, int64_t n, void* stream, gcmc_box** out) {
    g_last_error.clear();
    if (!out) return set_error(GCMC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate_desc(desc, n);
    if (rc) return rc;
    if (n > 0 && (!d_x || !d_y || !d_z)) return set_error(GCMC_ERR_INVALID_ARG, "coordinate arrays are NULL");
    hipStream_t s = (hipStream_t)stream;
    gcmc_box* box = new gcmc_box();
    memset(box, 0, sizeof(*box));
    for (int a = 0; a < 3; ++a) box->req_m[a] = desc->cell_m[a];
    for (int a = 0; a < desc->n_species * desc->n_species; ++a) {
        box->h_eps[a] = desc->eps[a];
        box->h_sig[a] = desc->sigma[a];
    }
    box->waves = 4;
    box->rows = 4;
    DevBox& B = box->d;
    std::vector<uint32_t> slots;
    if ((rc = setup_grid(B, desc, slots))) {
        free_box(box);
        return rc;
    }
    if (hipGetDevice(&box->device) != hipSuccess) {
        free_box(box);
        return set_error(GCMC_ERR_HIP, "no HIP device");
    }
    setup_params(B, desc);
    uint32_t* d_stab = nullptr;
    if (hipMalloc(&d_stab, slots.size() * sizeof(uint32_t)) != hipSuccess) {
        free_box(box);
        return set_error(GCMC_ERR_OOM, "box allocation failed");
    }
    B.stab = d_stab;
    if (hipMemcpy(d_stab, slots.data(), slots.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        free_box(box);
        return set_error(GCMC_ERR_HIP, "stencil upload failed");
    }
    if (hipMalloc(&B.pos, (size_t)B.max_n * sizeof(double4)) != hipSuccess ||
        hipMalloc(&B.count, (size_t)B.ncells * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&B.st, sizeof(BoxState)) != hipSuccess || hipMalloc(&box->d_desc, sizeof(DevBox)) != hipSuccess) {
        free_box(box);
        return set_error(GCMC_ERR_OOM, "box allocation failed");
    }
    // upload and count occupancy to size the cells
    k_reset_state<<<1, 1, 0, s>>>(B.st, n, 0.0, 0.0, 0);
    if (n > 0) k_upload<<<grid_for(n), 256, 0, s>>>(B, d_x, d_y, d_z, d_species, n);
    k_fill_i32<<<grid_for(B.ncells), 256, 0, s>>>(B.count, B.ncells, 0);
    if (n > 0) k_count<<<std::min(grid_for(n), kCountBlocks), 256, 0, s>>>(B, n);
    BoxState h;
    if ((rc = read_state(box, &h, s))) {
        free_box(box);
        return rc;
    }
    if (h.error) {
        free_box(box);
        return set_error(GCMC_ERR_INVALID_ARG, "coordinates must lie in [0, L) and species in [0, n_species)");
    }
    const int32_t cap = desc->cell_cap > 0 ? desc->cell_cap : auto_cap(h.maxcount);
    if (h.maxcount > cap) {
        free_box(box);
        return set_error(GCMC_ERR_CELL_OVERFLOW, "cell_cap smaller than the densest cell");
    }
    if ((rc = alloc_cells(box, cap)) || (rc = bin_particles(box, n, s, false, 0.0, 0.0)) ||
        (rc = read_state(box, &h, s))) {
        free_box(box);
        return rc;
    }
    if (h.error) {
        free_box(box);
        return set_error(h.error, "binning failed");
    }
    if ((rc = sync_desc(box))) {
        free_box(box);
        return rc;
    }
    *out = box;
    return GCMC_OK;
}

int gcmc_box_destroy(gcmc_box* box) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    (void)hipDeviceSynchronize();
    free_box(box);
    return GCMC_OK;
}

int gcmc_box_get_info(const gcmc_box* box, gcmc_box_info* info) {
    if (!box || !info) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    for (int a = 0; a < 3; ++a) {
        info->cell_m[a] = box->d.M[a];
        info->span[a] = box->d.span[a];
        info->inv_s[a] = box->d.invS[a];
    }
    info->cell_cap = box->d.cap;
    info->n_species = box->d.ns;
    info->n_cells = box->d.ncells;
    info->max_n = box->d.max_n;
    info->n_stencil = box->d.nstencil;
    info->pad = 0;
    return GCMC_OK;
}

int gcmc_cell_build(gcmc_box* box, int32_t new_cap, void* stream) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    if (new_cap < 0) return set_error(GCMC_ERR_INVALID_ARG, "new_cap must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = read_state(box, &h, s);
    if (rc) return rc;
    // a cell overflow and a wait past its bound both stop the chain before a move, every
    // earlier move committed: the rebuilt box resumes there
    if (h.error && h.error != GCMC_ERR_CELL_OVERFLOW && h.error != GCMC_ERR_INTERNAL)
        return set_error(GCMC_ERR_POISONED, "box holds a latched error that a rebuild does not clear");
    if (new_cap > 0 && new_cap != box->d.cap) {
        if ((rc = alloc_cells(box, new_cap))) return rc;
    }
    k_clear_rebuild_errors<<<1, 1, 0, s>>>(box->d.st);
    // keep N, running energy and the error move counter; re-bin
    const int64_t n = h.n;
    if ((rc = bin_particles(box, n, s, true, h.u_pair, h.w_pair))) return rc;
    if ((rc = read_state(box, &h, s))) return rc;
    if ((rc = sync_desc(box))) return rc;
    if (h.maxcount > box->d.cap) return set_error(GCMC_ERR_CELL_OVERFLOW, "cell_cap smaller than the densest cell");
    return GCMC_OK;
}

int gcmc_set_positions(gcmc_box* box, const double* d_x, const double* d_y, const double* d_z, int64_t n,
                       void* stream) {
    if (!box || ((!d_x || !d_y || !d_z) && n > 0)) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = read_state(box, &h, s);
    if (rc) return rc;
    if (h.error) return set_error(GCMC_ERR_POISONED, "box holds a latched error");
    if (n != h.n) return set_error(GCMC_ERR_INVALID_ARG, "n must equal the box's particle count");
    // species are kept: copy them out of the records first
    int32_t* sp = nullptr;
    if (h.n > 0) {
        GCMC_HIP(hipMallocAsync((void**)&sp, (size_t)h.n * sizeof(int32_t), s));
        k_get_particles<<<grid_for(h.n), 256, 0, s>>>(box->d, nullptr, nullptr, nullptr, sp);
        k_upload<<<grid_for(h.n), 256, 0, s>>>(box->d, d_x, d_y, d_z, sp, h.n);
        GCMC_HIP(hipFreeAsync(sp, s));
    }
    if ((rc = read_state(box, &h, s))) return rc;
    if (h.error) return set_error(GCMC_ERR_INVALID_ARG, "coordinates must lie in [0, L)");
    // the running energy and virial no longer describe the configuration
    const double nan = std::nan("");
    if ((rc = bin_particles(box, h.n, s, true, nan, nan))) return rc;
    if ((rc = read_state(box, &h, s))) return rc;
    if (h.error) return set_error(h.error, "re-binning overflowed a cell; rebuild with a larger cell_cap");
    return GCMC_OK;
}

int gcmc_set_params(gcmc_box* box, const double* h_eps, const double* h_sigma) {
    if (!box || !h_eps || !h_sigma) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    const int ns = box->d.ns;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            if (h_eps[a * ns + b] != h_eps[b * ns + a] || h_sigma[a * ns + b] != h_sigma[b * ns + a])
                return set_error(GCMC_ERR_INVALID_ARG, "eps/sigma tables must be symmetric");
            if (!(h_sigma[a * ns + b] > 0.0) || !(h_eps[a * ns + b] >= 0.0))
                return set_error(GCMC_ERR_INVALID_ARG, "need sigma > 0 and eps >= 0");
        }
    gcmc_box_desc d;
    memset(&d, 0, sizeof d);
    for (int a = 0; a < 3; ++a) d.L[a] = box->d.L[a];
    d.rc = sqrt(box->d.rc2);
    d.beta = box->d.beta;
    d.mu = box->d.mu;
    d.lambda3 = box->d.lambda3;
    d.max_disp = box->d.max_disp;
    d.p_disp = box->d.p_disp;
    d.n_species = ns;
    d.eps = h_eps;
    d.sigma = h_sigma;
    d.seed = box->d.seed;
    d.box_id = box->d.box_id;
    d.max_n = box->d.max_n;
    GCMC_HIP(hipDeviceSynchronize());
    setup_params(box->d, &d);
    box->d.rc2 = d.rc * d.rc;
    for (int a = 0; a < ns * ns; ++a) {
        box->h_eps[a] = h_eps[a];
        box->h_sig[a] = h_sigma[a];
    }
    // the running energy and virial belong to the old force field
    k_set_running<<<1, 1>>>(box->d.st, std::nan(""), std::nan(""));
    GCMC_HIP(hipGetLastError());
    GCMC_HIP(hipDeviceSynchronize());
    return sync_desc(box);
}

int gcmc_box_set_wait_limit(gcmc_box* box, int32_t polls) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    GCMC_HIP(hipDeviceSynchronize());
    box->d.wait_limit = polls;
    return sync_desc(box);
}

int gcmc_box_rescale(gcmc_box* box, const double* h_L, double* d_U, void* stream) {
    if (!box || !h_L || !d_U) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    DevBox& B = box->d;
    const double rc = sqrt(B.rc2);
    for (int a = 0; a < 3; ++a) {
        if (!(h_L[a] > 0.0) || !std::isfinite(h_L[a])) return set_error(GCMC_ERR_INVALID_ARG, "box edges must be positive");
        if (rc > 0.5 * h_L[a]) return set_error(GCMC_ERR_INVALID_ARG, "rc > L/2 breaks the minimum image");
    }
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc_ = read_state(box, &h, s);
    if (rc_) return rc_;
    if (h.error) return set_error(GCMC_ERR_POISONED, "box holds a latched error");
    const int64_t old_cells = B.ncells;
    // energies at the old volume
    if ((rc_ = ensure_scratch(box, total_partials_needed(B, h.maxcount, false, h.n)))) return rc_;
    int r = launch_total(B, box->d_desc, h.maxcount, false, nullptr, box->scratch, box->scratch_len, d_U + 2, s, h.n);
    if (r) return set_error(GCMC_ERR_INVALID_ARG, "scratch too small");
    // the new grid (the box's rule for cells per axis) and force-field constants
    gcmc_box_desc d;
    memset(&d, 0, sizeof d);
    for (int a = 0; a < 3; ++a) {
        d.L[a] = h_L[a];
        d.cell_m[a] = box->req_m[a];
    }
    d.rc = rc;
    d.beta = B.beta;
    d.mu = B.mu;
    d.lambda3 = B.lambda3;
    d.max_disp = B.max_disp;
    d.p_disp = B.p_disp;
    d.n_species = B.ns;
    d.eps = box->h_eps;
    d.sigma = box->h_sig;
    d.seed = B.seed;
    d.box_id = B.box_id;
    d.max_n = B.max_n;
    DevBox N2 = B;
    std::vector<uint32_t> slots;
    if ((rc_ = setup_grid(N2, &d, slots))) return rc_;
    setup_params(N2, &d);
    N2.rc2 = B.rc2;
    // From here on the box changes; a failure leaves it poisoned.
    GCMC_HIP(hipStreamSynchronize(s));
    uint32_t* d_stab = nullptr;
    if (hipMalloc(&d_stab, slots.size() * sizeof(uint32_t)) != hipSuccess)
        return set_error(GCMC_ERR_OOM, "stencil table allocation failed");
    GCMC_HIP(hipMemcpy(d_stab, slots.data(), slots.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    (void)hipFree((void*)B.stab);
    N2.stab = d_stab;
    if (N2.ncells != B.ncells) {
        (void)hipFree(B.count);
        N2.count = nullptr;
        if (hipMalloc(&N2.count, (size_t)N2.ncells * sizeof(int32_t)) != hipSuccess) {
            B = N2;
            return set_error(GCMC_ERR_OOM, "cell counter allocation failed");
        }
    }
    if (h.n > 0)
        k_rescale<<<grid_for(h.n), 256, 0, s>>>(B, h.n, h_L[0] / B.L[0], h_L[1] / B.L[1], h_L[2] / B.L[2], h_L[0],
                                                h_L[1], h_L[2]);
    B = N2;
    // occupancy at the new grid; the capacity grows (by the creation rule) if the densest cell needs it
    // the running virial is NaN until gcmc_virial sets it at the new volume
    k_reset_state<<<1, 1, 0, s>>>(B.st, h.n, h.u_pair, std::nan(""), 1);
    k_fill_i32<<<grid_for(B.ncells), 256, 0, s>>>(B.count, B.ncells, 0);
    if (h.n > 0) k_count<<<std::min(grid_for(h.n), kCountBlocks), 256, 0, s>>>(B, h.n);
    BoxState h2;
    if ((rc_ = read_state(box, &h2, s))) return rc_;
    const int32_t cap = h2.maxcount > B.cap ? auto_cap(h2.maxcount) : B.cap;
    if (cap != B.cap || B.ncells != old_cells) {
        if ((rc_ = alloc_cells(box, cap))) return rc_;
    }
    if ((rc_ = bin_particles(box, h.n, s, true, h.u_pair, std::nan(""))) || (rc_ = read_state(box, &h2, s)))
        return rc_;
    if (h2.error) return set_error(h2.error, "re-binning failed");
    if ((rc_ = sync_desc(box))) return rc_;
    // energies at the new volume (the running pair energy is reset to U_pair)
    if ((rc_ = ensure_scratch(box, total_partials_needed(B, h2.maxcount, false, h.n)))) return rc_;
    r = launch_total(B, box->d_desc, h2.maxcount, false, nullptr, box->scratch, box->scratch_len, d_U, s, h.n);
    if (r) return set_error(GCMC_ERR_INVALID_ARG, "scratch too small");
    GCMC_HIP(hipGetLastError());
    GCMC_HIP(hipStreamSynchronize(s));
    return GCMC_OK;
}

int gcmc_get_particles(gcmc_box* box, double* d_x, double* d_y, double* d_z, int32_t* d_species, int64_t* h_n,
                       void* stream) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = read_state(box, &h, s);
    if (rc) return rc;
    if (h.n > 0) k_get_particles<<<grid_for(h.n), 256, 0, s>>>(box->d, d_x, d_y, d_z, d_species);
    GCMC_HIP(hipGetLastError());
    GCMC_HIP(hipStreamSynchronize(s));
    if (h_n) *h_n = h.n;
    return GCMC_OK;
}

int gcmc_get_cells(gcmc_box* box, int32_t* d_cell_of, int32_t* d_count, int32_t* d_ids, void* stream) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    hipStream_t s = (hipStream_t)stream;
    k_get_cells<<<grid_for(box->d.ncells * box->d.cap), 256, 0, s>>>(box->d, d_cell_of, d_count, d_ids);
    GCMC_HIP(hipGetLastError());
    GCMC_HIP(hipStreamSynchronize(s));
    return GCMC_OK;
}

int gcmc_export_state(gcmc_box* box, double* d_x, double* d_y, double* d_z, int32_t* d_species, int64_t capacity,
                      gcmc_checkpoint* h_ck, void* stream) {
    if (!box || !h_ck) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = read_state(box, &h, s);
    if (rc) return rc;
    if ((d_x || d_y || d_z || d_species) && capacity < h.n)
        return set_error(GCMC_ERR_INVALID_ARG, "particle arrays shorter than N");
    if (h.n > 0 && (d_x || d_y || d_z || d_species)) {
        k_get_particles<<<grid_for(h.n), 256, 0, s>>>(box->d, d_x, d_y, d_z, d_species);
        GCMC_HIP(hipGetLastError());
        GCMC_HIP(hipStreamSynchronize(s));
    }
    memset(h_ck, 0, sizeof(*h_ck));
    h_ck->n = h.n;
    h_ck->u_pair = h.u_pair;
    h_ck->w_pair = h.w_pair;
    h_ck->counter = (uint64_t)h.counter;
    h_ck->moves = h.cum.moves;
    for (int t = 0; t < 3; ++t) {
        h_ck->attempts[t] = h.cum.att[t];
        h_ck->accepts[t] = h.cum.acc[t];
    }
    h_ck->sum_n = h.cum.sum_n;
    h_ck->sum_n2 = h.cum.sum_n2;
    h_ck->sum_u = h.cum.sum_u;
    h_ck->sum_w = h.cum.sum_w;
    h_ck->error = h.error;
    h_ck->error_move = h.error_move;
    return GCMC_OK;
}

int gcmc_import_state(gcmc_box* box, const double* d_x, const double* d_y, const double* d_z,
                      const int32_t* d_species, const gcmc_checkpoint* h_ck, void* stream) {
    if (!box || !h_ck) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    const int64_t n = h_ck->n;
    if (n < 0 || n > box->d.max_n) return set_error(GCMC_ERR_INVALID_ARG, "need 0 <= n <= max_n");
    if (n > 0 && (!d_x || !d_y || !d_z)) return set_error(GCMC_ERR_INVALID_ARG, "coordinate arrays are NULL");
    if (h_ck->error != GCMC_OK) return set_error(GCMC_ERR_INVALID_ARG, "a checkpoint with a latched error");
    hipStream_t s = (hipStream_t)stream;
    k_reset_state<<<1, 1, 0, s>>>(box->d.st, n, h_ck->u_pair, h_ck->w_pair, 0);
    if (n > 0) k_upload<<<grid_for(n), 256, 0, s>>>(box->d, d_x, d_y, d_z, d_species, n);
    BoxState h;
    int rc = read_state(box, &h, s);
    if (rc) return rc;
    if (h.error) return set_error(GCMC_ERR_INVALID_ARG, "coordinates must lie in [0, L) and species in range");
    if ((rc = bin_particles(box, n, s, false, h_ck->u_pair, h_ck->w_pair))) return rc;
    k_apply_checkpoint<<<1, 1, 0, s>>>(box->d.st, *h_ck);
    GCMC_HIP(hipGetLastError());
    if ((rc = read_state(box, &h, s))) return rc;
    if (h.error) return set_error(h.error, "binning overflowed a cell; rebuild with a larger cell_cap");
    return GCMC_OK;
}

int gcmc_clear_averages(gcmc_box* box, void* stream) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    k_clear_averages<<<1, 1, 0, (hipStream_t)stream>>>(box->d.st);
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_sync_status(gcmc_box* box) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    GCMC_HIP(hipDeviceSynchronize());
    BoxState h;
    GCMC_HIP(hipMemcpy(&h, box->d.st, sizeof(BoxState), hipMemcpyDeviceToHost));
    if (h.error) {
        char buf[160];
        snprintf(buf, sizeof buf, "box holds latched error %d raised at move %lld", h.error, (long long)h.error_move);
        return set_error(h.error, buf);
    }
    return GCMC_OK;
}

}  // extern "C"
