// Cell-list neighbour search under periodic boundary conditions.
//
// The paper updates its neighbour table with a binning method (Sec. IV.D) and
// stores it as the padded, per-pair-type tensor R_abc with a mask (Sec. III.A).
// Here the table is kept as one padded row per (atom, neighbour species b),
// nbr[atom][b][c] with `cap` slots per row, and a count per (b, atom) in place
// of the mask.  Atoms are renumbered in cell-major order so that the atoms a
// wave visits are spatially close and their neighbours share cache lines.
//
// Inclusion predicate (evaluated in FP64, every operation separately rounded):
//   w = x - L*floor(x/L) (then folded into [0, L)),
//   d = (w_j - w_i) + n*L per component, d2 = dx*dx + dy*dy + dz*dz,
//   keep (j, n) != (i, 0) when d2 < rlist*rlist.
#include "tmd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

// No fused multiply-adds anywhere in this file: the predicate must round every
// product and sum separately, like its FP64 definition.
#pragma clang fp contract(off)

namespace tmd {
namespace {

constexpr int kErrNonFinite = 1;
constexpr int kErrSpecies = 2;
constexpr int kErrCoincident = 4;

__device__ inline double wrap_exact(double x, double L) {
    double w = x - L * floor(x / L);
    if (w < 0.0) w = w + L;
    if (w >= L) w = w - L;
    return w;
}

__device__ inline int cell_coord(double w, double inv_cw, int nc) {
    int c = (int)(w * inv_cw);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

struct GridArgs {
    double L[3];
    double inv_cw[3];
    int nc[3];
    int reach[3];
};

__global__ void k_bin(int64_t n, const double* __restrict__ pos, const int32_t* __restrict__ species, int S,
                      GridArgs g, double* __restrict__ wpos, int32_t* __restrict__ cell_of,
                      int32_t* __restrict__ cell_rank, int32_t* __restrict__ cellcount,
                      int32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3];
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
        double x = pos[3 * i + a];
        if (!isfinite(x)) { bad = true; x = 0.0; }
        double w = wrap_exact(x, g.L[a]);
        wpos[3 * i + a] = w;
        c[a] = cell_coord(w, g.inv_cw[a], g.nc[a]);
    }
    if (bad) atomicOr(&flags[0], kErrNonFinite);
    int s = species[i];
    if (s < 0 || s >= S) atomicOr(&flags[0], kErrSpecies);
    int cell = (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
    cell_of[i] = cell;
    // Arrival order in the cell (k_sort_gather fixes the order).  Consecutive
    // lanes in one cell (atoms in lattice or trajectory order) form a run that
    // takes one atomic: its first lane adds the run length, and the run's lanes
    // take consecutive ranks.  The active lanes are a prefix of the wave.
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(cell, 1);
    const bool head = lane == 0 || prev != cell;
    const unsigned long long heads = __ballot(head), active = __ballot(true);
    const int h = 63 - __builtin_clzll(heads & ((2ull << lane) - 1));  // this lane's run head
    const unsigned long long after = heads & ~((2ull << h) - 1);       // heads past it
    const int end = after ? __builtin_ctzll(after) : 64 - __builtin_clzll(active);
    int base = 0;
    if (head) base = atomicAdd(&cellcount[cell], end - h);
    base = __shfl(base, h);
    cell_rank[i] = base + (lane - h);
}

// Exclusive scan by one block of 1024 threads over tiles of 1024 consecutive
// elements in[q * stride] (coalesced for stride 1); out[n] receives the total.
__device__ void block_exclusive_scan(int64_t n, const int32_t* __restrict__ in, int stride,
                                     int32_t* __restrict__ out, int out_stride) {
    __shared__ int32_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int32_t carry = 0;
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t q = base + t;
        const int32_t v = q < n ? in[q * stride] : 0;
        int32_t x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int32_t pre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int32_t s = wsum[w];
            pre += (w < wv) ? s : 0;
            tot += s;
        }
        if (q < n) out[q * out_stride] = carry + pre + x - v;
        carry += tot;
        __syncthreads();
    }
    if (t == 0) out[n * out_stride] = carry;
}

// Exclusive scan of the cell counts (cells are few: about N/14).
// Cell starts in three passes (any cell count): k_scan_tiles scans each tile
// of 1024 cells and records its total and the largest count; k_scan_tile_sums
// scans the tile totals in one workgroup; k_scan_add adds each tile's offset.
__global__ void __launch_bounds__(1024) k_scan_tiles(int64_t ncells, const int32_t* __restrict__ count,
                                                     int32_t* __restrict__ start, int32_t* __restrict__ tile_sum,
                                                     int32_t* __restrict__ max_occ) {
    __shared__ int32_t wsum[16], wmax[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t q = (int64_t)blockIdx.x * 1024 + t;
    const int32_t v = q < ncells ? count[q] : 0;
    int32_t x = v, m = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if (lane == 63) wsum[wv] = x;
    if (lane == 0) wmax[wv] = m;
    __syncthreads();
    int32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const int32_t sw = wsum[w];
        pre += (w < wv) ? sw : 0;
        tot += sw;
    }
    if (q < ncells) start[q] = pre + x - v;
    if (t == 0) {
        tile_sum[blockIdx.x] = tot;
        int32_t mm = wmax[0];
        for (int w = 1; w < 16; ++w) mm = max(mm, wmax[w]);
        atomicMax(max_occ, mm);
    }
}

__global__ void __launch_bounds__(1024) k_scan_tile_sums(int64_t ntiles, int32_t* __restrict__ tile_sum) {
    block_exclusive_scan(ntiles, tile_sum, 1, tile_sum, 1);
}

__global__ void k_scan_add(int64_t ncells, const int32_t* __restrict__ tile_off, int32_t* __restrict__ start) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < ncells) start[q] += tile_off[q >> 10];
    if (q == ncells) start[q] = tile_off[(ncells + 1023) >> 10];
}

// Per-species exclusive scans over the per-block species counts; the totals
// go to spcount[s] for the host.
__global__ void __launch_bounds__(1024) k_species_scan(int64_t nblk, int S, const int32_t* __restrict__ blkcnt,
                                                       int32_t* __restrict__ blkoff, int32_t* __restrict__ spcount) {
    for (int s = 0; s < S; ++s) {
        block_exclusive_scan(nblk, blkcnt + s, kMaxSpecies, blkoff + s, kMaxSpecies);
        __syncthreads();
        if (threadIdx.x == 0) spcount[s] = blkoff[nblk * kMaxSpecies + s];
        __syncthreads();
    }
}

__global__ void k_place(int64_t n, const int32_t* __restrict__ cell_of, const int32_t* __restrict__ cell_rank,
                        const int32_t* __restrict__ start, int32_t* __restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    order[start[cell_of[i]] + cell_rank[i]] = (int32_t)i;
}

// Sixteen lanes per cell (cells hold about 14 atoms at the list cutoff): the
// cell's atoms (in the arbitrary order the atomic placement left) are ranked by
// original index, which fixes a deterministic order, and each atom's wrapped
// position, image shift, species and cell are gathered straight to its sorted
// slot start[cell] + rank.  Fuller cells take several rounds of 16.
constexpr int kSortLanes = 16;
__global__ void __launch_bounds__(256) k_sort_gather(int64_t ncells, const int32_t* __restrict__ start,
                                                     const int32_t* __restrict__ order, const double* __restrict__ wpos,
                                                     const double* __restrict__ pos,
                                                     const int32_t* __restrict__ species, GridArgs g,
                                                     int32_t* __restrict__ perm, int32_t* __restrict__ shift,
                                                     double4* __restrict__ xs, int32_t* __restrict__ sp,
                                                     int32_t* __restrict__ cell_sorted) {
    const int lane = threadIdx.x % kSortLanes;
    const int64_t cell = (int64_t)blockIdx.x * (kBlock / kSortLanes) + threadIdx.x / kSortLanes;
    if (cell >= ncells) return;  // whole group
    const int lo = start[cell], m = start[cell + 1] - lo;
    for (int k0 = 0; k0 < m; k0 += kSortLanes) {
        const int k = k0 + lane;
        const int32_t v = k < m ? order[lo + k] : INT32_MAX;
        int r = 0;  // entries of the cell with a smaller original index
        for (int j0 = 0; j0 < m; j0 += kSortLanes) {
            const int32_t vj = j0 + lane < m ? order[lo + j0 + lane] : INT32_MAX;
            const int nj = min(kSortLanes, m - j0);
            for (int t = 0; t < nj; ++t) r += __shfl(vj, t, kSortLanes) < v ? 1 : 0;
        }
        if (k < m) {
            const int64_t p = lo + r;
            const int32_t i = v;
            perm[p] = i;
            double w[3];
            for (int a = 0; a < 3; ++a) {
                w[a] = wpos[3 * (int64_t)i + a];
                const double x = pos[3 * (int64_t)i + a];
                const double kk = isfinite(x) ? rint((w[a] - x) / g.L[a]) : 0.0;
                shift[3 * p + a] = (int32_t)kk;
            }
            xs[p] = make_double4(w[0], w[1], w[2], 0.0);
            sp[p] = species[i];
            cell_sorted[p] = (int32_t)cell;
        }
    }
}

// Rows of the list pruned to the cutoff at the current positions: each wave
// takes kPruneRows consecutive rows (row t = p * S + b) and issues the loads of
// all of them (counts, the first 64 entries and image words, then the
// neighbour positions) before it compacts any, so that a wave waits for a few
// memory round trips in total instead of a few per row; the rare entries past
// the first 64 of a row follow one 64-entry chunk at a time.  Kept entries
// keep their order.
constexpr int kPruneRows = 4;

// The full rows are read once and the pruned rows written once per step:
// streamed past the caches, which keep the neighbour positions.
__device__ __forceinline__ int32_t ld_stream(const int32_t* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(int32_t* p, int32_t v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ bool prune_keep(double xi, double yi, double zi, const double* xj, int32_t im, double L0,
                                           double L1, double L2, double rc2) {
    int nx, ny, nz;
    unpack_img(im, nx, ny, nz);
    const double dx = (xj[0] - xi) + (double)nx * L0;
    const double dy = (xj[1] - yi) + (double)ny * L1;
    const double dz = (xj[2] - zi) + (double)nz * L2;
    return (dx * dx + dy * dy) + dz * dz < rc2;
}

__global__ void __launch_bounds__(256) k_prune(int64_t n, int S, int cap, double rc2, const double4* __restrict__ xs,
                                               double L0, double L1, double L2, const int32_t* __restrict__ nbr,
                                               const int32_t* __restrict__ img, const int32_t* __restrict__ cnt,
                                               int32_t* __restrict__ pnbr, int32_t* __restrict__ pimg,
                                               int32_t* __restrict__ pcnt, const int32_t* __restrict__ gate) {
    if (gate && gate[0] == 0) return;  // uniform: the pruned rows are still valid
    const int lane = threadIdx.x & 63;
    const int64_t rows = n * S;
    // wave-uniform row range: counts and centre positions come in scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * kPruneRows;
    if (t0 >= rows) return;  // whole wave
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int c[kPruneRows];
    int64_t pr[kPruneRows];  // atom of each row (its species b = t - p * S)
    int32_t q[kPruneRows], im[kPruneRows];
    double xj[kPruneRows][3];
    {
        int64_t p = t0 / S;
        int b = (int)(t0 - p * S);
#pragma unroll
        for (int r = 0; r < kPruneRows; ++r) {
            const int64_t t = t0 + r;
            const bool ok = t < rows;
            pr[r] = ok ? p : 0;
            c[r] = ok ? cnt[(int64_t)b * n + p] : 0;
            if (++b == S) {
                b = 0;
                ++p;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kPruneRows; ++r) {
        q[r] = lane < c[r] ? ld_stream(nbr + (t0 + r) * cap + lane) : 0;
        im[r] = lane < c[r] ? ld_stream(img + (t0 + r) * cap + lane) : 0;
    }
#pragma unroll
    for (int r = 0; r < kPruneRows; ++r)
        if (lane < c[r]) {
            const double* x = reinterpret_cast<const double*>(xs + q[r]);
            xj[r][0] = x[0];
            xj[r][1] = x[1];
            xj[r][2] = x[2];
        }
#pragma unroll
    for (int r = 0; r < kPruneRows; ++r) {
        const int64_t t = t0 + r;
        const int64_t p = pr[r];
        const double4 xi = xs[p];
        const bool keep = lane < c[r] && prune_keep(xi.x, xi.y, xi.z, xj[r], im[r], L0, L1, L2, rc2);
        const unsigned long long m = __ballot(keep);
        if (keep) {
            const int slot = (int)__popcll(m & below);
            st_stream(pnbr + t * cap + slot, q[r]);
            st_stream(pimg + t * cap + slot, im[r]);
        }
        int kept = (int)__popcll(m);
        for (int k0 = 64; k0 < c[r]; k0 += 64) {  // c[r] is uniform: whole-wave loop
            const int k = k0 + lane;
            bool kk = false;
            int32_t qq = 0, ii = 0;
            if (k < c[r]) {
                qq = nbr[t * cap + k];
                ii = img[t * cap + k];
                kk = prune_keep(xi.x, xi.y, xi.z, reinterpret_cast<const double*>(xs + qq), ii, L0, L1, L2, rc2);
            }
            const unsigned long long mm = __ballot(kk);
            if (kk) {
                const int slot = kept + (int)__popcll(mm & below);
                pnbr[t * cap + slot] = qq;
                pimg[t * cap + slot] = ii;
            }
            kept += (int)__popcll(mm);
        }
        if (lane == 0 && t < rows) pcnt[(t - p * S) * n + p] = kept;
    }
}

// One thread: does this evaluation need new pruned rows (see PruneGate)?
__global__ void k_prune_gate(const unsigned long long* __restrict__ maxd2, double* __restrict__ state,
                             int32_t* __restrict__ flag, int force, double half_margin) {
    if (threadIdx.x != 0) return;
    const double d = sqrt(__longlong_as_double((long long)maxd2[0]));
    if (force || !(d + state[0] < half_margin)) {
        flag[0] = 1;
        state[0] = force ? 0.0 : d;  // a forced prune follows a build: no displacement yet
    } else {
        flag[0] = 0;
    }
}

// Per 256-atom block of the sorted order, the count of each species (invalid
// species fail the build on the host and are not counted); scanned over
// blocks by k_species_scan.
__global__ void __launch_bounds__(256) k_species_blocks(int64_t n, const int32_t* __restrict__ sp,
                                                        int32_t* __restrict__ blkcnt) {
    __shared__ int32_t wc[kBlock / 64][kMaxSpecies];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = p < n ? sp[p] : -1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int b = 0; b < kMaxSpecies; ++b) {
        const unsigned long long m = __ballot(s == b);
        if (lane == 0) wc[wv][b] = (int32_t)__popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < kMaxSpecies) {
        int32_t tot = 0;
        for (int w = 0; w < kBlock / 64; ++w) tot += wc[w][threadIdx.x];
        blkcnt[(int64_t)blockIdx.x * kMaxSpecies + threadIdx.x] = tot;
    }
}

struct FillArgs {
    GridArgs g;
    int64_t n;
    int S, cap;
    double rl2;
    const double4* xs;
    const int32_t* sp;
    const int32_t* cell_sorted;
    const int32_t* cellstart;
    int32_t* nbr;
    int32_t* img;
    int32_t* cnt;
    int32_t* flags;
    bool narrow;       // 3x3x3 stencil: entries record their stencil offset code
};

__device__ inline int floor_div(int a, int b) {
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Largest atom count of a cell block of B0 x B1 x B2 cells plus its one-cell
// periodic halo into *out: waves stride over the blocks (lanes over a block's
// halo cells); one atomic per workgroup.
constexpr int kHaloMaxGroups = 256;
__global__ void __launch_bounds__(256) k_halo_max(GridArgs g, int3 A, int64_t nbA, int3 B, int64_t nbB, int3 C,
                                                  int64_t nbC, const int32_t* __restrict__ start,
                                                  int32_t* __restrict__ out) {
    __shared__ int32_t wmax[3][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // largest atom count of one block of shape S plus its one-cell halo
    auto largest = [&](int3 S, int64_t nblocks) {
        const int nb0 = (g.nc[0] + S.x - 1) / S.x, nb1 = (g.nc[1] + S.y - 1) / S.y;
        const int HX = S.x + 2, HY = S.y + 2, nh = HX * HY * (S.z + 2);
        int best = 0;
        for (int64_t blk = (int64_t)blockIdx.x * (kBlock / 64) + wv; blk < nblocks;
             blk += (int64_t)gridDim.x * (kBlock / 64)) {
            const int x0 = (int)(blk % nb0) * S.x, y0 = (int)((blk / nb0) % nb1) * S.y,
                      z0 = (int)(blk / ((int64_t)nb0 * nb1)) * S.z;
            int c = 0;
            for (int h = lane; h < nh; h += 64) {
                const int x = x0 - 1 + h % HX, y = y0 - 1 + (h / HX) % HY, z = z0 - 1 + h / (HX * HY);
                const int wx = x - floor_div(x, g.nc[0]) * g.nc[0];
                const int wy = y - floor_div(y, g.nc[1]) * g.nc[1];
                const int wz = z - floor_div(z, g.nc[2]) * g.nc[2];
                const int cell = (wz * g.nc[1] + wy) * g.nc[0] + wx;
                c += start[cell + 1] - start[cell];
            }
            for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
            best = max(best, c);
        }
        return best;
    };
    const int bestA = largest(A, nbA), bestB = largest(B, nbB), bestC = largest(C, nbC);
    if (lane == 0) {
        wmax[0][wv] = bestA;
        wmax[1][wv] = bestB;
        wmax[2][wv] = bestC;
    }
    __syncthreads();
    if (threadIdx.x < 3) {  // out[0 .. 2]: shapes A, B, C
        int m = wmax[threadIdx.x][0];
        for (int w = 1; w < kBlock / 64; ++w) m = max(m, wmax[threadIdx.x][w]);
        atomicMax(out + threadIdx.x, m);
    }
}


// Systems of at most this many atoms have every workgroup of k_fill stage all
// positions in LDS (32 KB): their cells are few and crowded, so each thread
// walks hundreds of candidates, which the lanes of one cell then read from
// LDS at one address instead of from L2.  The per-thread FP64 tests still
// bound such a launch: a few workgroups run the whole list serially.
constexpr int kFillLdsAtoms = 1024;

// One thread per atom (cell-major order): scan the stencil of cells within
// `reach` (periodic images folded in), append accepted neighbours to the
// list of their species.
template <bool kLds>
__global__ void __launch_bounds__(256) k_fill(FillArgs a) {
    __shared__ double4 xs_lds[kLds ? kFillLdsAtoms : 1];
    if constexpr (kLds) {
        for (int64_t i = threadIdx.x; i < a.n; i += blockDim.x) xs_lds[i] = a.xs[i];
        __syncthreads();
    }
    auto pos = [&](int64_t i) -> double4 {
        if constexpr (kLds)
            return xs_lds[i];
        else
            return a.xs[i];
    };
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const GridArgs& g = a.g;
    const double4 xi = pos(p);
    const int cell = a.cell_sorted[p];
    const int cx = cell % g.nc[0];
    const int cy = (cell / g.nc[0]) % g.nc[1];
    const int cz = cell / (g.nc[0] * g.nc[1]);
    int cnt[kMaxSpecies];
#pragma unroll
    for (int b = 0; b < kMaxSpecies; ++b) cnt[b] = 0;
    bool coincident = false;
    int o = 0;  // stencil offset index in traversal order
    for (int oz = -g.reach[2]; oz <= g.reach[2]; ++oz) {
        const int zz = cz + oz;
        const int nz = floor_div(zz, g.nc[2]);
        const int wz = zz - nz * g.nc[2];
        const double sz = (double)nz * g.L[2];
        for (int oy = -g.reach[1]; oy <= g.reach[1]; ++oy) {
            const int yy = cy + oy;
            const int ny = floor_div(yy, g.nc[1]);
            const int wy = yy - ny * g.nc[1];
            const double sy = (double)ny * g.L[1];
            for (int ox = -g.reach[0]; ox <= g.reach[0]; ++ox) {
                const int xx = cx + ox;
                const int nx = floor_div(xx, g.nc[0]);
                const int wx = xx - nx * g.nc[0];
                const double sx = (double)nx * g.L[0];
                const int c2 = (wz * g.nc[1] + wy) * g.nc[0] + wx;
                const int lo = a.cellstart[c2], hi = a.cellstart[c2 + 1];
                const bool zero_img = (nx == 0 && ny == 0 && nz == 0);
                // stencil offset code of this cell (0..26), stored with each entry when the stencil is 3x3x3
                const int ocode = a.narrow ? stencil_bits(o) : 255;
                ++o;
                // candidates in batches of 4: all position loads issued first
                for (int q0 = lo; q0 < hi; q0 += 4) {
                    double4 xj[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) xj[j] = pos(min(q0 + j, hi - 1));
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int q = q0 + j;
                        if (q >= hi || (zero_img && q == p)) continue;
                        const double dx = (xj[j].x - xi.x) + sx;
                        const double dy = (xj[j].y - xi.y) + sy;
                        const double dz = (xj[j].z - xi.z) + sz;
                        const double d2 = (dx * dx + dy * dy) + dz * dz;
                        if (!(d2 < a.rl2)) continue;
                        if (d2 == 0.0) coincident = true;
                        const int b = a.sp[q];
                        if (b < 0 || b >= a.S) continue;  // reported by k_bin; never index with it
                        int k = 0;
#pragma unroll
                        for (int bb = 0; bb < kMaxSpecies; ++bb)
                            if (bb == b) { k = cnt[bb]; cnt[bb] = k + 1; }
                        if (k < a.cap) {
                            // row-major: this thread's entries are consecutive addresses
                            const int64_t off = (p * a.S + b) * a.cap + k;
                            a.nbr[off] = q;
                            a.img[off] = pack_img(nx, ny, nz, ocode);
                        }
                    }
                }
            }
        }
    }
    int mx = 0;
#pragma unroll
    for (int b = 0; b < kMaxSpecies; ++b) {
        if (b < a.S) a.cnt[(int64_t)b * a.n + p] = min(cnt[b], a.cap);
        mx = max(mx, cnt[b]);
    }
    if (mx > a.cap) atomicMax(&a.flags[1], mx);
    if (coincident) atomicOr(&a.flags[0], kErrCoincident);
}

constexpr int kMaxCellAtoms = 64;
constexpr int kMaxCandidates = 27 * kMaxCellAtoms;

// One wave per cell (stencils of at most 64 cells, cells of at most 64 atoms,
// at most kMaxCandidates candidates).  Each round the wave holds 64
// candidates of the cell's stencil, in the same order as k_fill visits them
// (stencil cell, then atom), and tests them with the same FP64 predicate
// against every atom of the cell in turn (the atom's position is a uniform,
// scalar load).  An atom's accepted candidates are compacted with one ballot
// (split by species with per-round species masks) and written to its rows as
// one contiguous run per species, so the list is identical to k_fill's while
// every load and store of the wave is coalesced.
// Image of cell coordinate c (in -1 .. n) when the stencil reaches one cell.
__device__ __forceinline__ int near_image(int c, int n) { return c < 0 ? -1 : (c >= n ? 1 : 0); }

template <int SMAX, bool NARROW>  // a.S <= SMAX; NARROW: 3x3x3 stencil
__global__ void __launch_bounds__(256) k_fill_cells(FillArgs a, int64_t ncells) {
    // per wave: stencil cell of every candidate, and the cell's own positions
    __shared__ uint8_t s_cell[kBlock / 64][kMaxCandidates];
    __shared__ double s_xi[kBlock / 64][3][kMaxCellAtoms];
    __shared__ int32_t s_len[kBlock / 64][kMaxCellAtoms][SMAX];  // running row lengths
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t cell = (int64_t)blockIdx.x * (kBlock / 64) + wv;
    if (cell >= ncells) return;  // whole wave
    const GridArgs& g = a.g;
    const int cx = (int)(cell % g.nc[0]), cy = (int)((cell / g.nc[0]) % g.nc[1]),
              cz = (int)(cell / ((int64_t)g.nc[0] * g.nc[1]));
    const int a0 = __builtin_amdgcn_readfirstlane(a.cellstart[cell]);
    const int natoms = __builtin_amdgcn_readfirstlane(a.cellstart[cell + 1]) - a0;
    if (natoms == 0) return;  // nothing to list (and a0 may equal n)
    if (natoms > kMaxCellAtoms) {  // the host reruns the build with k_fill
        if (lane == 0) atomicOr(&a.flags[2], 1);
        return;
    }
    const int rx = NARROW ? 1 : g.reach[0], ry = NARROW ? 1 : g.reach[1], rz = NARROW ? 1 : g.reach[2];
    const int wx = 2 * rx + 1, wy = 2 * ry + 1, wz = 2 * rz + 1;
    const int ns = wx * wy * wz;
    if (lane < natoms) {
        const double4 x = a.xs[a0 + lane];
        s_xi[wv][0][lane] = x.x;
        s_xi[wv][1][lane] = x.y;
        s_xi[wv][2][lane] = x.z;
    }
    // every stencil cell inside the box (no periodic image): uniform
    const bool interior = cx - rx >= 0 && cx + rx < g.nc[0] && cy - ry >= 0 && cy + ry < g.nc[1] &&
                          cz - rz >= 0 && cz + rz < g.nc[2];
    // stencil cell of this lane (traversal order: z outer, x inner)
    int first = 0, count = 0;
    if (lane < ns) {
        const int ox = lane % wx - rx, oy = (lane / wx) % wy - ry, oz = lane / (wx * wy) - rz;
        const int xx = cx + ox, yy = cy + oy, zz = cz + oz;
        const int nx = floor_div(xx, g.nc[0]), ny = floor_div(yy, g.nc[1]), nz = floor_div(zz, g.nc[2]);
        const int c2 = ((zz - nz * g.nc[2]) * g.nc[1] + (yy - ny * g.nc[1])) * g.nc[0] + (xx - nx * g.nc[0]);
        first = a.cellstart[c2];
        count = a.cellstart[c2 + 1] - first;
    }
    int pre = count;  // inclusive scan over the stencil cells
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(pre, off);
        if (lane >= off) pre += y;
    }
    const int total = __shfl(pre, 63);
    pre -= count;  // exclusive
    if (total > kMaxCandidates) {  // the host reruns the build with k_fill
        if (lane == 0) atomicOr(&a.flags[2], 1);
        return;
    }
    // candidate -> stencil cell table: stencil cell s owns candidates [pre_s, pre_s + count_s)
    for (int j = 0; j < count; ++j) s_cell[wv][pre + j] = (uint8_t)lane;
    for (int t = lane; t < natoms * SMAX; t += 64) (&s_len[wv][0][0])[t] = 0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool coincident = false;
    for (int k0 = 0; k0 < total; k0 += 64) {
        const int k = k0 + lane;
        const bool valid = k < total;
        const int sk = valid ? (int)s_cell[wv][k] : 0;
        const int ox = sk % wx - rx, oy = (sk / wx) % wy - ry, oz = sk / (wx * wy) - rz;
        const int nx = NARROW ? near_image(cx + ox, g.nc[0]) : floor_div(cx + ox, g.nc[0]);
        const int ny = NARROW ? near_image(cy + oy, g.nc[1]) : floor_div(cy + oy, g.nc[1]);
        const int nz = NARROW ? near_image(cz + oz, g.nc[2]) : floor_div(cz + oz, g.nc[2]);
        const double sx = (double)nx * g.L[0];
        const double sy = (double)ny * g.L[1];
        const double sz = (double)nz * g.L[2];
        // every lane takes part in both shuffles (a shuffle from a lane that
        // is inactive in a branch yields undefined data); select afterwards
        const int first_sk = __shfl(first, sk);
        const int pre_sk = __shfl(pre, sk);
        const int q = valid ? first_sk + (k - pre_sk) : a0;
        const double4 xj = a.xs[q];
        const int bq = valid ? a.sp[q] : -1;
        const bool okq = valid && bq >= 0 && bq < a.S;
        const bool zero_img = (nx == 0 && ny == 0 && nz == 0);
        const int32_t word = pack_img(nx, ny, nz, a.narrow ? stencil_bits(sk) : 255);
        // candidates of each species this round, and this lane's own species' mask
        unsigned long long spm[SMAX], mine = 0;
#pragma unroll
        for (int b = 0; b < SMAX; ++b) {
            spm[b] = __ballot(okq && bq == b);
            if (bq == b) mine = spm[b];
        }
        // this lane's entry offset inside a (atom, species) row block
        const int lane_row = okq ? bq * a.cap : 0;
        const unsigned long long mine_below = mine & below;
        const unsigned long long mine_above = mine & ~below & ~(1ull << lane);
        // row lengths of the cell's atoms for this lane's species, in LDS: each
        // lane reads its species' length of atom i, and the last accepted lane
        // of each species stores the new length
        int32_t* len = &s_len[wv][0][okq ? bq : 0];
        // SHIFT: some candidate of the stencil lies in a periodic image.  A
        // cell whose whole stencil is inside the box adds only +0.0 image
        // shifts, which change no distance, so they are left out there.
        auto test_atoms = [&](auto shift) {
            constexpr bool SHIFT = decltype(shift)::value;
            // row blocks of the cell's atoms, advanced by one atom's rows per step
            const int64_t row_step = (int64_t)a.S * a.cap;
            char* nrow = reinterpret_cast<char*>(a.nbr + (int64_t)a0 * row_step);
            char* irow = reinterpret_cast<char*>(a.img + (int64_t)a0 * row_step);
            for (int i = 0; i < natoms; ++i, nrow += 4 * row_step, irow += 4 * row_step) {
                const int p = a0 + i;
                const double4 xi = make_double4(s_xi[wv][0][i], s_xi[wv][1][i], s_xi[wv][2][i], 0.0);
                double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
                if constexpr (SHIFT) {
                    dx = dx + sx;
                    dy = dy + sy;
                    dz = dz + sz;
                }
                const double d2 = (dx * dx + dy * dy) + dz * dz;
                const bool acc = okq && !((SHIFT ? zero_img : true) && q == p) && d2 < a.rl2;
                if (acc && d2 == 0.0) coincident = true;
                const unsigned long long m = __builtin_amdgcn_ballot_w64(acc);
                if (!m) continue;
                if (acc) {
                    const int c = len[i * SMAX] + (int)__popcll(m & mine_below);
                    // past the capacity the build fails and is redone with a larger
                    // one, so those entries only need to stay inside their row
                    const uint32_t boff = 4u * (uint32_t)(lane_row + min(c, a.cap - 1));
                    *reinterpret_cast<int32_t*>(nrow + boff) = q;
                    *reinterpret_cast<int32_t*>(irow + boff) = word;
                    if ((m & mine_above) == 0) len[i * SMAX] = c + 1;  // last of its species
                }
            }
        };
        if (interior)
            test_atoms(std::false_type{});
        else
            test_atoms(std::true_type{});
    }
    int mx = 0;
    if (lane < natoms) {
        const int p = a0 + lane;
#pragma unroll
        for (int b = 0; b < SMAX; ++b) {
            if (b >= a.S) break;
            const int c = s_len[wv][lane][b];
            a.cnt[(int64_t)b * a.n + p] = min(c, a.cap);
            mx = max(mx, c);
        }
    }
    if (mx > a.cap) atomicMax(&a.flags[1], mx);
    if (coincident) atomicOr(&a.flags[0], kErrCoincident);
}

// Atoms grouped by species in sorted order, without atomics: block offsets
// from k_species_scan, wave offsets from the block's ballots, lane rank.
__global__ void k_species_place(int64_t n, int S, const int32_t* __restrict__ sp, const int32_t* __restrict__ spcount,
                                const int32_t* __restrict__ blkoff, int32_t* __restrict__ sp_idx) {
    __shared__ int32_t wc[kBlock / 64][kMaxSpecies];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = p < n ? sp[p] : -1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long mine = 0;
    for (int b = 0; b < kMaxSpecies; ++b) {
        const unsigned long long m = __ballot(s == b);
        if (lane == 0) wc[wv][b] = (int32_t)__popcll(m);
        if (s == b) mine = m;
    }
    __syncthreads();
    if (s >= 0 && s < S) {  // an invalid species fails the build on the host; it is not placed
        int32_t woff = 0;
        for (int w = 0; w < wv; ++w) woff += wc[w][s];
        int64_t base = 0;  // atoms of the species before s
        for (int b = 0; b < s; ++b) base += spcount[b];
        sp_idx[base + blkoff[(int64_t)blockIdx.x * kMaxSpecies + s] + woff + (int)__popcll(mine & below)] =
            (int32_t)p;
    }
}

__global__ void k_export(int64_t n, int S, int cap, const int32_t* __restrict__ perm, const int32_t* __restrict__ nbr,
                         const int32_t* __restrict__ img, const int32_t* __restrict__ cnt, int32_t* __restrict__ onbr,
                         int32_t* __restrict__ oimg, int32_t* __restrict__ ocnt) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = perm[p];
    for (int b = 0; b < S; ++b) {
        const int c = cnt[(int64_t)b * n + p];
        ocnt[i * S + b] = c;
        for (int k = 0; k < cap; ++k) {
            const int64_t src = (p * S + b) * cap + k;
            const int64_t dst = (i * S + b) * cap + k;
            if (k < c) {
                onbr[dst] = perm[nbr[src]];
                int nx, ny, nz;
                unpack_img(img[src], nx, ny, nz);
                oimg[3 * dst] = nx;
                oimg[3 * dst + 1] = ny;
                oimg[3 * dst + 2] = nz;
            } else {
                onbr[dst] = -1;
                oimg[3 * dst] = oimg[3 * dst + 1] = oimg[3 * dst + 2] = 0;
            }
        }
    }
}

__global__ void k_refresh(int64_t n, const double* __restrict__ pos, const int32_t* __restrict__ perm,
                          const int32_t* __restrict__ shift, double L0, double L1, double L2,
                          double4* __restrict__ xs) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = perm[p];
    const double x = pos[3 * i] + (double)shift[3 * p] * L0;
    const double y = pos[3 * i + 1] + (double)shift[3 * p + 1] * L1;
    const double z = pos[3 * i + 2] + (double)shift[3 * p + 2] * L2;
    xs[p] = make_double4(x, y, z, 0.0);
}

// Sum and maximum of the row counts: grid-stride, one pair of atomics per
// workgroup (a pair per wave made 2 M rows cost 0.75 ms of serialised atomics).
constexpr int kStatsGroups = 256;
__global__ void __launch_bounds__(256) k_count_stats(int64_t total, const int32_t* __restrict__ cnt,
                                                     unsigned long long* __restrict__ sum, int32_t* __restrict__ mx) {
    __shared__ unsigned long long ws[kBlock / 64];
    __shared__ int32_t wm[kBlock / 64];
    unsigned long long s = 0;
    int m = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int v = cnt[q];
        s += (unsigned long long)v;
        m = max(m, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        m = max(m, __shfl_xor(m, off));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        ws[wv] = s;
        wm[wv] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            s += ws[w];
            m = max(m, wm[w]);
        }
        atomicAdd(sum, s);
        atomicMax(mx, m);
    }
}

inline unsigned grid_for(int64_t n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

}  // namespace

tmd_status launch_build_neighbors(tmd_context* ctx, const tmd_system_view* sys, double rlist, tmd_nlist* nl,
                                  int32_t* required_capacity) {
    const int64_t n = sys->n_atoms;
    GridArgs g;
    int64_t ncells = 1;
    for (int a = 0; a < 3; ++a) {
        const double L = sys->box[a];
        int nc = (int)std::floor(L / (rlist * (1.0 + 1e-9)));
        nc = std::max(1, std::min(nc, 1 << 20));
        g.L[a] = L;
        g.nc[a] = nc;
        ncells *= nc;
    }
    // Keep the cell count proportional to the atom count (sparse boxes).
    const int64_t max_cells = std::max<int64_t>(64, 4 * n);
    while (ncells > max_cells) {
        int a = 0;
        for (int b = 1; b < 3; ++b)
            if (g.nc[b] > g.nc[a]) a = b;
        ncells /= g.nc[a];
        g.nc[a] = std::max(1, g.nc[a] / 2);
        ncells *= g.nc[a];
    }
    for (int a = 0; a < 3; ++a) {
        g.inv_cw[a] = (double)g.nc[a] / g.L[a];
        g.reach[a] = g.nc[a] == 1 ? (int)std::ceil(rlist / g.L[a]) : 1;
        if (g.reach[a] > 100)
            return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "box edge far smaller than the cutoff");
    }
    hipError_t e = hipSuccess;
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    const bool narrow = g.reach[0] == 1 && g.reach[1] == 1 && g.reach[2] == 1;
    if (nl->cellstart_cap < ncells + 1) {
        if (nl->cellstart) (void)hipFree(nl->cellstart);
        nl->cellstart = nullptr;
        nl->cellstart_cap = 0;
        TMD_HIP(ctx, hipMalloc((void**)&nl->cellstart, sizeof(int32_t) * (ncells + 1)));
        nl->cellstart_cap = ncells + 1;
    }
    int32_t* cellstart = nl->cellstart;
    double* wpos = (double*)ctx->ws.get("nb.wpos", sizeof(double) * 3 * n, &e);
    int32_t* cell_of = (int32_t*)ctx->ws.get("nb.cell_of", sizeof(int32_t) * n, &e);
    int32_t* cell_sorted = (int32_t*)ctx->ws.get("nb.cell_sorted", sizeof(int32_t) * n, &e);
    int32_t* order = (int32_t*)ctx->ws.get("nb.order", sizeof(int32_t) * n, &e);
    int32_t* cellcount = (int32_t*)ctx->ws.get("nb.cellcount", sizeof(int32_t) * (ncells + 1), &e);
    int32_t* tiles = (int32_t*)ctx->ws.get("nb.tiles", sizeof(int32_t) * ((ncells + 1023) / 1024 + 1), &e);
    int32_t* cell_rank = (int32_t*)ctx->ws.get("nb.cell_rank", sizeof(int32_t) * n, &e);
    int32_t* blkcnt = (int32_t*)ctx->ws.get("nb.blkcnt", sizeof(int32_t) * kMaxSpecies * nblk, &e);
    int32_t* blkoff = (int32_t*)ctx->ws.get("nb.blkoff", sizeof(int32_t) * kMaxSpecies * (nblk + 1), &e);
    int32_t* flags = (int32_t*)ctx->ws.get("nb.flags", sizeof(int32_t) * 64, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "neighbour workspace allocation");
    hipStream_t st = ctx->stream;
    int32_t* spcount = flags + 8;
    TMD_HIP(ctx, hipMemsetAsync(cellcount, 0, sizeof(int32_t) * (ncells + 1), st));
    TMD_HIP(ctx, hipMemsetAsync(flags, 0, sizeof(int32_t) * 64, st));

    {
        ProfScope ps_(ctx, "nb_bin");
        k_bin<<<grid_for(n), kBlock, 0, st>>>(n, sys->pos, sys->species, nl->S, g, wpos, cell_of, cell_rank,
                                               cellcount, flags);
    }
    {
        ProfScope ps_(ctx, "nb_scan");
        const int64_t ntiles = (ncells + 1023) / 1024;
        k_scan_tiles<<<(unsigned)ntiles, 1024, 0, st>>>(ncells, cellcount, cellstart, tiles, flags + 4);
        k_scan_tile_sums<<<1, 1024, 0, st>>>(ntiles, tiles);
        k_scan_add<<<grid_for(ncells + 1), kBlock, 0, st>>>(ncells, tiles, cellstart);
    }
    if (narrow) {
        // the block shapes the work order prefers, clamped to the grid
        auto shape = [&](const int* B) {
            return make_int3(std::min(B[0], g.nc[0]), std::min(B[1], g.nc[1]), std::min(B[2], g.nc[2]));
        };
        auto count = [&](int3 S) {
            return (int64_t)((g.nc[0] + S.x - 1) / S.x) * ((g.nc[1] + S.y - 1) / S.y) * ((g.nc[2] + S.z - 1) / S.z);
        };
        const int3 A = shape(kBlockShape), B = shape(kBlockShape2), C = shape(kBlockShape3);
        const int64_t nbA = count(A), nbB = count(B), nbC = count(C);
        ProfScope ps_(ctx, "nb_halo_max");
        const int64_t groups =
            std::min<int64_t>(kHaloMaxGroups, (std::max({nbA, nbB, nbC}) + kBlock / 64 - 1) / (kBlock / 64));
        k_halo_max<<<(unsigned)groups, kBlock, 0, st>>>(g, A, nbA, B, nbB, C, nbC, cellstart, flags + 5);
    }
    {
        ProfScope ps_(ctx, "nb_place");
        k_place<<<grid_for(n), kBlock, 0, st>>>(n, cell_of, cell_rank, cellstart, order);
    }
    {
        ProfScope ps_(ctx, "nb_sort");
        k_sort_gather<<<(unsigned)((ncells + kBlock / kSortLanes - 1) / (kBlock / kSortLanes)), kBlock, 0, st>>>(
            ncells, cellstart, order, wpos, sys->pos, sys->species, g, nl->perm, nl->shift, nl->xs, nl->sp,
            cell_sorted);
    }
    {
        ProfScope ps_(ctx, "nb_species_blocks");
        k_species_blocks<<<grid_for(n), kBlock, 0, st>>>(n, nl->sp, blkcnt);
    }
    {
        ProfScope ps_(ctx, "nb_species_scan");
        k_species_scan<<<1, 1024, 0, st>>>(nblk, nl->S, blkcnt, blkoff, spcount);
    }
    {
        ProfScope ps_(ctx, "nb_species");
        k_species_place<<<grid_for(n), kBlock, 0, st>>>(n, nl->S, nl->sp, spcount, blkoff, nl->sp_idx);
    }
    FillArgs fa;
    fa.g = g;
    fa.n = n;
    fa.S = nl->S;
    fa.cap = nl->cap;
    fa.rl2 = rlist * rlist;
    fa.xs = nl->xs;
    fa.sp = nl->sp;
    fa.cell_sorted = cell_sorted;
    fa.cellstart = cellstart;
    fa.nbr = nl->nbr;
    fa.img = nl->img;
    fa.cnt = nl->cnt;
    fa.flags = flags;
    fa.narrow = narrow;
    const int stencil_cells = (2 * g.reach[0] + 1) * (2 * g.reach[1] + 1) * (2 * g.reach[2] + 1);
    const bool by_cell = stencil_cells <= 64;
    if (by_cell) {
        ProfScope ps_(ctx, "nb_fill");
        const unsigned grid = (unsigned)((ncells + kBlock / 64 - 1) / (kBlock / 64));
        using FillFn = void (*)(FillArgs, int64_t);
        FillFn fn;
        if (nl->S == 1)
            fn = narrow ? k_fill_cells<1, true> : k_fill_cells<1, false>;
        else if (nl->S == 2)
            fn = narrow ? k_fill_cells<2, true> : k_fill_cells<2, false>;
        else if (nl->S <= 4)
            fn = narrow ? k_fill_cells<4, true> : k_fill_cells<4, false>;
        else
            fn = narrow ? k_fill_cells<kMaxSpecies, true> : k_fill_cells<kMaxSpecies, false>;
        fn<<<grid, kBlock, 0, st>>>(fa, ncells);
    } else {
        ProfScope ps_(ctx, "nb_fill");
        if (n <= kFillLdsAtoms)
            k_fill<true><<<grid_for(n), kBlock, 0, st>>>(fa);
        else
            k_fill<false><<<grid_for(n), kBlock, 0, st>>>(fa);
    }
    TMD_HIP(ctx, hipGetLastError());
    TMD_HIP(ctx, hipMemcpyAsync(ctx->h_flags, flags, sizeof(int32_t) * 64, hipMemcpyDeviceToHost, st));
    TMD_HIP(ctx, hipStreamSynchronize(st));
    if (by_cell && (ctx->h_flags[2] & 1)) {
        // a cell holds more atoms than one wave can track: per-atom fill instead
        {
            ProfScope ps_(ctx, "nb_fill");
            if (n <= kFillLdsAtoms)
                k_fill<true><<<grid_for(n), kBlock, 0, st>>>(fa);
            else
                k_fill<false><<<grid_for(n), kBlock, 0, st>>>(fa);
        }
        TMD_HIP(ctx, hipGetLastError());
        TMD_HIP(ctx, hipMemcpyAsync(ctx->h_flags, flags, sizeof(int32_t) * 64, hipMemcpyDeviceToHost, st));
        TMD_HIP(ctx, hipStreamSynchronize(st));
    }
    const int32_t errs = ctx->h_flags[0];
    if (errs & kErrSpecies) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "species index outside [0, n_species)");
    if (errs & kErrNonFinite) return fail(ctx, TMD_ERR_NUMERICAL, "non-finite atomic position");
    if (errs & kErrCoincident) return fail(ctx, TMD_ERR_NUMERICAL, "two atoms at distance zero");
    const int32_t need = ctx->h_flags[1];
    if (need > nl->cap) {
        if (required_capacity) *required_capacity = need;
        nl->built = false;
        return fail(ctx, TMD_ERR_CAPACITY, "neighbour list capacity " + std::to_string(nl->cap) +
                                               " too small; need " + std::to_string(need));
    }
    if (required_capacity) *required_capacity = need;
    int64_t off = 0;
    for (int s = 0; s < nl->S; ++s) {
        nl->sp_count[s] = ctx->h_flags[8 + s];
        nl->sp_off[s] = off;
        off += nl->sp_count[s];
    }
    nl->sp_off[nl->S] = off;
    nl->n = n;
    nl->rlist = rlist;
    nl->ncells = ncells;
    nl->max_occ = ctx->h_flags[4];
    nl->halo_max = narrow ? ctx->h_flags[5] : -1;
    nl->halo_max2 = narrow ? ctx->h_flags[6] : -1;
    nl->halo_max3 = narrow ? ctx->h_flags[7] : -1;
    nl->narrow = narrow;
    for (int a = 0; a < 3; ++a) {
        nl->box[a] = sys->box[a];
        nl->nc[a] = g.nc[a];
        nl->reach[a] = g.reach[a];
    }
    nl->built = true;
    ++nl->build_id;
    return launch_work_order(ctx, nl);
}

namespace {

tmd_status reserve_pruned(tmd_context* ctx, tmd_nlist* nl) {
    if (nl->pnbr) return TMD_OK;
    const size_t lst = (size_t)nl->nmax * nl->S * nl->cap;
    hipError_t e = hipMalloc((void**)&nl->pnbr, 4 * lst);
    if (e == hipSuccess) e = hipMalloc((void**)&nl->pimg, 4 * lst);
    if (e == hipSuccess) e = hipMalloc((void**)&nl->pcnt, 4 * (size_t)nl->nmax * nl->S);
    if (e == hipSuccess) e = hipMalloc((void**)&nl->prune_state, 16);
    if (e != hipSuccess) {
        for (void** q : {(void**)&nl->pnbr, (void**)&nl->pimg, (void**)&nl->pcnt, (void**)&nl->prune_state}) {
            if (*q) (void)hipFree(*q);
            *q = nullptr;
        }
        return hip_fail(ctx, e, "pruned neighbour list allocation");
    }
    nl->prune_flag = reinterpret_cast<int32_t*>(nl->prune_state + 1);
    return TMD_OK;
}

tmd_status prune_rows(tmd_context* ctx, tmd_nlist* nl, double r, const int32_t* gate) {
    const int64_t rows = nl->n * nl->S;
    {
        ProfScope ps_(ctx, "prune");
        const int64_t waves = (rows + kPruneRows - 1) / kPruneRows;
        k_prune<<<(unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, ctx->stream>>>(
            nl->n, nl->S, nl->cap, r * r, nl->xs, nl->box[0], nl->box[1], nl->box[2], nl->nbr, nl->img, nl->cnt,
            nl->pnbr, nl->pimg, nl->pcnt, gate);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace

tmd_status reserve_pruned_rows(tmd_context* ctx, tmd_nlist* nl) { return reserve_pruned(ctx, nl); }

tmd_status launch_prune(tmd_context* ctx, tmd_nlist* nl, double rcut) {
    tmd_status st = reserve_pruned(ctx, nl);
    if (st != TMD_OK) return st;
    nl->pruned_margin = -1.0;
    return prune_rows(ctx, nl, rcut * (1.0 + 1e-6), nullptr);
}

tmd_status launch_prune_gated(tmd_context* ctx, tmd_nlist* nl, double rcut, const PruneGate& g) {
    if (!g.maxd2 || !(g.margin > 0.0)) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "prune gate without displacements");
    tmd_status st = reserve_pruned(ctx, nl);
    if (st != TMD_OK) return st;
    const int force = (nl->pruned_build_id != nl->build_id || nl->pruned_margin != g.margin) ? 1 : 0;
    k_prune_gate<<<1, 64, 0, ctx->stream>>>(g.maxd2, nl->prune_state, nl->prune_flag, force, 0.5 * g.margin);
    TMD_HIP(ctx, hipGetLastError());
    nl->pruned_build_id = nl->build_id;
    nl->pruned_margin = g.margin;
    return prune_rows(ctx, nl, rcut + g.margin, nl->prune_flag);
}

tmd_status launch_refresh_positions(tmd_context* ctx, const tmd_system_view* sys, const tmd_nlist* nl) {
    const int64_t n = nl->n;
    {
        ProfScope ps_(ctx, "refresh");
        k_refresh<<<grid_for(n), kBlock, 0, ctx->stream>>>(n, sys->pos, nl->perm, nl->shift, sys->box[0], sys->box[1],
                                                            sys->box[2], nl->xs);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status reserve_nlist_workspace(tmd_context* ctx, int64_t n, int S) {
    (void)S;
    hipError_t e = hipSuccess;
    const int64_t nblk = (n + kBlock - 1) / kBlock, cells = std::max<int64_t>(64, 4 * n) + 1;
    (void)ctx->ws.get("nb.wpos", sizeof(double) * 3 * n, &e);
    (void)ctx->ws.get("nb.cell_of", sizeof(int32_t) * n, &e);
    (void)ctx->ws.get("nb.cell_sorted", sizeof(int32_t) * n, &e);
    (void)ctx->ws.get("nb.order", sizeof(int32_t) * n, &e);
    (void)ctx->ws.get("nb.cellcount", sizeof(int32_t) * cells, &e);
    (void)ctx->ws.get("nb.tiles", sizeof(int32_t) * ((cells + 1023) / 1024 + 1), &e);
    (void)ctx->ws.get("wo.count", sizeof(int32_t) * cells, &e);
    (void)ctx->ws.get("nb.cell_rank", sizeof(int32_t) * n, &e);
    (void)ctx->ws.get("nb.blkcnt", sizeof(int32_t) * kMaxSpecies * nblk, &e);
    (void)ctx->ws.get("nb.blkoff", sizeof(int32_t) * kMaxSpecies * (nblk + 1), &e);
    (void)ctx->ws.get("nb.flags", sizeof(int32_t) * 64, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "neighbour workspace allocation");
    return TMD_OK;
}

size_t nlist_workspace_bytes(int64_t n) {
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    const size_t cells = (size_t)std::max<int64_t>(64, 4 * n) + 1;
    return (size_t)n * 40 + 8 * cells + 4 * (cells / 1024 + 2) + 8 * (size_t)kMaxSpecies * (nblk + 1) + 512;
}

tmd_status launch_nlist_stats(tmd_context* ctx, const tmd_nlist* nl, int64_t* total_pairs, int32_t* max_row) {
    hipError_t e = hipSuccess;
    void* buf = ctx->ws.get("nb.stats", 64, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "stats workspace");
    unsigned long long* sum = (unsigned long long*)buf;
    int32_t* mx = (int32_t*)((char*)buf + 8);
    const int64_t total = (int64_t)nl->S * nl->n;
    TMD_HIP(ctx, hipMemsetAsync(buf, 0, 16, ctx->stream));
    {
        ProfScope ps_(ctx, "nb_stats");
        k_count_stats<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(kStatsGroups, grid_for(total))), kBlock, 0,
                        ctx->stream>>>(total, nl->cnt, sum, mx);
    }
    TMD_HIP(ctx, hipGetLastError());
    TMD_HIP(ctx, hipMemcpyAsync(ctx->h_flags, buf, 16, hipMemcpyDeviceToHost, ctx->stream));
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long s;
    std::memcpy(&s, ctx->h_flags, 8);
    if (total_pairs) *total_pairs = (int64_t)s;
    if (max_row) *max_row = ctx->h_flags[2];
    return TMD_OK;
}

tmd_status launch_export_nlist(tmd_context* ctx, const tmd_nlist* nl, int32_t* nbr, int32_t* img, int32_t* cnt) {
    const int64_t n = nl->n;
    {
        ProfScope ps_(ctx, "nb_export");
        k_export<<<grid_for(n), kBlock, 0, ctx->stream>>>(n, nl->S, nl->cap, nl->perm, nl->nbr, nl->img, nl->cnt, nbr,
                                                           img, cnt);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd
