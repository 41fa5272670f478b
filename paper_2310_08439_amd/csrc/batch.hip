// Energy and forces of several systems in one launch chain: the systems'
// resident neighbour lists are merged into one list over the concatenation of
// their atoms (each system's atoms a segment, padded to a multiple of 256 so
// that no workgroup of the adjoint spans two systems), and the descriptor,
// MLP and adjoint kernels run once over the whole of it.  A pair's image
// shift uses the box of its centre atom's system (a per-atom box), the forces
// go back to each system's own output array, and the energy and virial are
// summed per system, in FP64 with Neumaier compensation in a fixed order.
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

// Segment holding combined atom g (segments are ordered by offset).
__device__ __forceinline__ int find_segment(const BatchSeg* __restrict__ segs, int nseg, int64_t g) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Positions (wrapped as the system's own list has them), boxes, row counts and
// rows of the merged list; neighbour indices are shifted by the segment offset.
// Padding atoms get no rows.
__global__ void k_batch_merge(const BatchSeg* __restrict__ segs, int nseg, int64_t N, int S, int cap,
                              double4* __restrict__ xs, double4* __restrict__ boxes, int32_t* __restrict__ nbr,
                              int32_t* __restrict__ img, int32_t* __restrict__ cnt) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const BatchSeg& sg = segs[find_segment(segs, nseg, g)];
    const int64_t p = g - sg.off;
    if (p >= sg.n) {
        xs[g] = make_double4(0.0, 0.0, 0.0, 0.0);
        boxes[g] = make_double4(1.0, 1.0, 1.0, 0.0);
        for (int b = 0; b < S; ++b) cnt[(int64_t)b * N + g] = 0;
        return;
    }
    const int64_t i = sg.perm[p];
    xs[g] = make_double4(sg.pos[3 * i] + (double)sg.shift[3 * p] * sg.L[0],
                         sg.pos[3 * i + 1] + (double)sg.shift[3 * p + 1] * sg.L[1],
                         sg.pos[3 * i + 2] + (double)sg.shift[3 * p + 2] * sg.L[2], 0.0);
    boxes[g] = make_double4(sg.L[0], sg.L[1], sg.L[2], 0.0);
    for (int b = 0; b < S; ++b) {
        const int c = sg.cnt[(int64_t)b * sg.n + p];
        cnt[(int64_t)b * N + g] = c;
        const int32_t* sn = sg.nbr + (p * S + b) * sg.cap;
        const int32_t* si = sg.img + (p * S + b) * sg.cap;
        int32_t* dn = nbr + (g * S + b) * cap;
        int32_t* di = img + (g * S + b) * cap;
        for (int k = 0; k < c; ++k) {
            dn[k] = sn[k] + (int32_t)sg.off;
            di[k] = si[k];
        }
    }
}

// Atoms grouped by species over all segments: species b holds segment 0's
// species-b atoms, then segment 1's, and so on.
__global__ void k_batch_species(const BatchSeg* __restrict__ segs, int nseg, int64_t N, int S,
                                int32_t* __restrict__ sp_idx) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const BatchSeg& sg = segs[find_segment(segs, nseg, g)];
    const int64_t k = g - sg.off;  // position in the segment's own grouping
    if (k >= sg.n) return;
    int b = 0;
    while (b + 1 < S && sg.sp_off[b + 1] <= k) ++b;
    sp_idx[sg.dst_off[b] + (k - sg.sp_off[b])] = (int32_t)(sg.off + sg.sp_idx[k]);
}

// Fixed-point forces to each system's output in its own atom order.
__global__ void k_batch_scatter(const BatchSeg* __restrict__ segs, int nseg, int64_t N,
                                const unsigned long long* __restrict__ Fq) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const BatchSeg& sg = segs[find_segment(segs, nseg, g)];
    const int64_t p = g - sg.off;
    if (p >= sg.n) return;
    const int64_t i = sg.perm[p];
    constexpr double inv = 1.0 / kForceFixedScale;
#pragma unroll
    for (int c = 0; c < 3; ++c) sg.forces[3 * i + c] = (float)((double)(long long)Fq[3 * g + c] * inv);
}

// Block s: totals[7 s .. 7 s + 6] = (sum E_i, virial xx yy zz xy xz yz) of
// segment s, from its atoms' E_i and its adjoint workgroups' virial partials
// (vir_atoms combined atoms per partial); fixed per-thread ranges and a fixed
// reduction tree.
__global__ void __launch_bounds__(256) k_batch_totals(const BatchSeg* __restrict__ segs, const float* __restrict__ Ei,
                                                      const double* __restrict__ vir, int vir_atoms,
                                                      double* __restrict__ totals) {
    __shared__ double red_s[7][4], red_c[7][4];
    const BatchSeg& sg = segs[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Comp acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = Comp{0.0, 0.0};
    for (int64_t p = threadIdx.x; p < sg.n; p += 256) comp_add(acc[0], (double)Ei[sg.off + p]);
    const int64_t v0 = sg.off / vir_atoms, v1 = (sg.off + sg.npad) / vir_atoms;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256)
#pragma unroll
        for (int j = 0; j < 6; ++j)
            acc[1 + j] = comp_merge(acc[1 + j], Comp{vir[v * kVirDoubles + 2 * j], vir[v * kVirDoubles + 2 * j + 1]});
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        for (int off = 32; off > 0; off >>= 1) {
            const Comp o{__shfl_xor(acc[j].s, off), __shfl_xor(acc[j].c, off)};
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
        totals[7 * blockIdx.x + threadIdx.x] = r.s + r.c;
    }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

tmd_status launch_batch_merge(tmd_context* ctx, const BatchSeg* segs, int nseg, tmd_nlist* vnl, double4* boxes) {
    {
        ProfScope ps_(ctx, "batch_merge");
        k_batch_merge<<<grid_of(vnl->n), kBlock, 0, ctx->stream>>>(segs, nseg, vnl->n, vnl->S, vnl->cap, vnl->xs, boxes,
                                                                    vnl->nbr, vnl->img, vnl->cnt);
        k_batch_species<<<grid_of(vnl->n), kBlock, 0, ctx->stream>>>(segs, nseg, vnl->n, vnl->S, vnl->sp_idx);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_batch_finalize(tmd_context* ctx, const BatchSeg* segs, int nseg, int64_t N,
                                 const unsigned long long* Fq, const float* Ei, const double* vir, int vir_atoms,
                                 double* totals) {
    {
        ProfScope ps_(ctx, "batch_finalize");
        k_batch_scatter<<<grid_of(N), kBlock, 0, ctx->stream>>>(segs, nseg, N, Fq);
        k_batch_totals<<<(unsigned)nseg, 256, 0, ctx->stream>>>(segs, Ei, vir, vir_atoms, totals);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd
