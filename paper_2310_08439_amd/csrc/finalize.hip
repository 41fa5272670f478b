// Output assembly: forces and atomic energies back to the caller's atom order,
// total energy and virial reduced in FP64 with Neumaier compensation in a fixed
// order (one block, fixed per-thread ranges, fixed tree), so the totals are
// reproducible run to run.
#include "tmd_internal.h"

namespace tmd {
namespace {

struct Comp {
    double s, c;
};

__device__ __forceinline__ void comp_add(Comp& a, double x) {
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x;
    else a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ Comp comp_merge(Comp a, Comp b) {
    comp_add(a, b.s);
    a.c += b.c;
    return a;
}

// Forces (fixed point, 32 fractional bits) and atomic energies back to the
// caller's atom order: F = q 2^-32, exact in FP64, then rounded to FP32.
__global__ void k_scatter_out(int64_t n, const int32_t* __restrict__ perm, const float* __restrict__ Ei,
                              const unsigned long long* __restrict__ Fq, float* __restrict__ atom_energy,
                              float* __restrict__ forces) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = perm[p];
    constexpr double inv = 1.0 / kForceFixedScale;
    forces[3 * i + 0] = (float)((double)(long long)Fq[3 * p + 0] * inv);
    forces[3 * i + 1] = (float)((double)(long long)Fq[3 * p + 1] * inv);
    forces[3 * i + 2] = (float)((double)(long long)Fq[3 * p + 2] * inv);
    if (atom_energy) atom_energy[i] = Ei[p];
}

constexpr int kPartBlocks = 256;

// Fixed-order block reduction of 7 compensated sums: butterfly inside each
// wave, then a serial pass over the 4 waves.  Result valid in thread 0..6.
__device__ void block_merge(Comp (&acc)[7], double (*red_s)[4], double (*red_c)[4], Comp* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        for (int off = 32; off > 0; off >>= 1) {
            Comp o{__shfl_xor(acc[j].s, off), __shfl_xor(acc[j].c, off)};
            acc[j] = (lane & off) ? comp_merge(o, acc[j]) : comp_merge(acc[j], o);
        }
        if (lane == 0) {
            red_s[j][wv] = acc[j].s;
            red_c[j][wv] = acc[j].c;
        }
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        Comp r{0.0, 0.0};
        for (int w = 0; w < 4; ++w) r = comp_merge(r, Comp{red_s[threadIdx.x][w], red_c[threadIdx.x][w]});
        out[threadIdx.x] = r;
    }
}

// Stage 1: block b sums a contiguous slice of Ei and of the virial block
// partials with coalesced, thread-strided reads.
__global__ void __launch_bounds__(256) k_partials(int64_t n, const float* __restrict__ Ei, int64_t nvir,
                                                  const double* __restrict__ vir, double* __restrict__ part) {
    __shared__ double red_s[7][4], red_c[7][4];
    __shared__ Comp res[7];
    Comp acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = Comp{0.0, 0.0};
    const int64_t per = (n + kPartBlocks - 1) / kPartBlocks;
    const int64_t lo = blockIdx.x * per, hi = min<int64_t>(n, lo + per);
    // unrolled so that a chunk's loads are in flight together (the sums keep
    // their order: each thread adds its values in index order)
#pragma unroll 8
    for (int64_t p = lo + threadIdx.x; p < hi; p += 256) comp_add(acc[0], (double)Ei[p]);
    const int64_t pv = (nvir + kPartBlocks - 1) / kPartBlocks;
    const int64_t vlo = blockIdx.x * pv, vhi = min<int64_t>(nvir, vlo + pv);
    for (int64_t b = vlo + threadIdx.x; b < vhi; b += 256)
#pragma unroll
        for (int j = 0; j < 6; ++j)
            acc[1 + j] = comp_merge(acc[1 + j], Comp{vir[b * kVirDoubles + 2 * j], vir[b * kVirDoubles + 2 * j + 1]});
    block_merge(acc, red_s, red_c, res);
    if (threadIdx.x < 7) {
        part[(blockIdx.x * 7 + threadIdx.x) * 2] = res[threadIdx.x].s;
        part[(blockIdx.x * 7 + threadIdx.x) * 2 + 1] = res[threadIdx.x].c;
    }
}

// Stage 2: totals[0] = sum Ei; totals[1..6] = virial (xx, yy, zz, xy, xz, yz).
__global__ void __launch_bounds__(256) k_totals(const double* __restrict__ part, double* __restrict__ totals) {
    __shared__ double red_s[7][4], red_c[7][4];
    __shared__ Comp res[7];
    Comp acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j)
        acc[j] = Comp{part[(threadIdx.x * 7 + j) * 2], part[(threadIdx.x * 7 + j) * 2 + 1]};
    block_merge(acc, red_s, red_c, res);
    if (threadIdx.x < 7) totals[threadIdx.x] = res[threadIdx.x].s + res[threadIdx.x].c;
}

// out[perm[p] or p][f] = in[p][column of f at the padded radial functions]
// for the model's features f = (b Kabi + k)(M+1) + m.
__global__ void k_permute_rows(int64_t n, int Fabi, int F, int Kabi, int K, int M1, const int32_t* __restrict__ perm,
                               const float* __restrict__ in, float* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * Fabi) return;
    const int64_t p = idx / Fabi;
    const int f = (int)(idx - p * Fabi);
    const int per_b = Kabi * M1, b = f / per_b, r = f - b * per_b;
    const int fi = (b * K + r / M1) * M1 + r % M1;
    out[(perm ? (int64_t)perm[p] : p) * Fabi + f] = in[p * F + fi];
}

}  // namespace

tmd_status launch_finalize(tmd_context* ctx, const tmd_nlist* nl, const float* Ei, const unsigned long long* Fs,
                           const double* vir_partials, int nvir, float* atom_energy, float* forces, double* totals7,
                           double* part) {
    static_assert(finalize_part_doubles() == kPartBlocks * 14, "partials of the two-stage reduction");
    const int64_t n = nl->n;
    {
        ProfScope ps_(ctx, "scatter_out");
        k_scatter_out<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, nl->perm, Ei, Fs,
                                                                                         atom_energy, forces);
    }
    {
        ProfScope ps_(ctx, "partials");
        k_partials<<<kPartBlocks, 256, 0, ctx->stream>>>(n, Ei, nvir, vir_partials, part);
    }
    {
        ProfScope ps_(ctx, "totals");
        k_totals<<<1, kPartBlocks, 0, ctx->stream>>>(part, totals7);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_permute_rows(tmd_context* ctx, const tmd_nlist* nl, const float* in, const tmd_model* m, float* out) {
    const int64_t total = nl->n * m->Fabi;
    {
        ProfScope ps_(ctx, "permute_rows");
        k_permute_rows<<<(unsigned)((total + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
            nl->n, m->Fabi, m->F, m->Kabi, m->K, m->M + 1, nl->perm, in, out);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_compact_features(tmd_context* ctx, int64_t n, const float* in, int F, int Fabi, int K, int Kabi,
                                   int M1, float* out) {
    const int64_t total = n * Fabi;
    if (total == 0) return TMD_OK;
    k_permute_rows<<<(unsigned)((total + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, Fabi, F, Kabi, K, M1,
                                                                                         nullptr, in, out);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd
