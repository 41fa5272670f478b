// Descriptor (forward) and adjoint (backward) kernels of the TensorMD path.
//
// Forward (Sec. III.A, eqns G_radial_tensor_form, tensor_formalism,
// sigma_function): for centre atom a and neighbour species b,
//   P[b][k][d] = sum_c h_k(R_c) M_d(u_c),  S[b][k][m] = sum_{d in m} T_dm P^2,
//   G[b][k][m] = sqrt(S) (m = 0) or S (m > 0).
// Backward (eqns dP_abkd, U_abck, F1_abcx, F2_abcx): with sigma' = dE/dS,
//   P'[b][k][d] = 2 T_dm sigma'[b][k][m(d)] P[b][k][d],
//   U_ck = sum_d P'_kd M_cd,  V_cd = sum_k P'_kd h_ck,
//   g_c = dE/dD_c = (sum_k U_ck h'_ck) u_c + (1/R)(sum_d V_cd grad_u M_d - u_c sum_d ord(d) V_cd M_cd),
// the last bracket being F2 = V M' with M' = dM/dD evaluated on the fly from
// u and R (the paper's memory-saving choice for F2), and the first term F1 =
// U H' R'.  Forces: F_a += g_c, F_j -= g_c (ScatterSum); virial W -= D (x) g.
//
// Thread mapping: one thread per (centre atom, chunk of KC radial functions);
// the K/KC chunk threads of an atom are adjacent lanes.  Each thread keeps its
// P (or P') tile of KC x D values in registers and streams the atom's
// neighbours from its row of the row-major list, recomputing the pair
// geometry.  The only per-pair data in HBM is the list itself; the descriptor
// pass also stores P (K x D floats per atom and element) so that the adjoint
// pass can form P' without a second neighbour sweep.
// Per-pair force partials of the chunks are summed with lane shuffles.
//
// Radial functions: direct (Gaussian x cosine cutoff, exp2 recurrence on a
// uniform grid) or, in the TAB instantiations, a cubic-Hermite table lookup
// with the cutoff folded in (Sec. III.B's tabulated H and H'): per pair one
// contiguous run of KC coefficient quadruples, no transcendental.
#include "tmd_internal.h"
#include "tensor_ops.h"

#include <algorithm>
#include <type_traits>

namespace tmd {
namespace {

using namespace ops;

struct PathArgs {
    int64_t n;
    int S, K, F, cap, nch_log2;
    float rc2, half_inv_rc, pi_over_rc;
    int rec;
    float rec_a, rec_b, rec_c;
    float rec_m2eta, rec_delta;  // uniform grid: -2 eta and the centre spacing Delta
    float rec_c4;                // rec_c^16, the step of four radial functions (when rec4)
    // radial table (TAB kernels): [(tab_n + 1)][K] cubic coefficients, spacing 1/tab_inv
    const float4* tab;
    float tab_inv;
    int tab_n;
    double L[3];
    // per-atom box edges (x, y, z) when the atoms of several systems share one
    // list (tmd_energy_forces_batch); nullptr: every atom's box is L
    const double4* boxes;
    const double4* xs;
    const int32_t* nbr;
    const int32_t* img;
    const int32_t* cnt;
    // work slot -> sorted atom (nullptr: identity); P is stored by work slot
    const int32_t* wperm;
    const float* mu;
    const float* eta;
    // forward output / backward input; with Gb non-null the forward output is
    // stored there as the bits of (__bf16)G instead (the BF16 MLP's operand)
    float* G;
    uint16_t* Gb;
    const float* dG;
    // P written by the forward pass (if non-null) and read back by the
    // adjoint: [S][K][DR][n] by work slot (VALU kernels), or, for the
    // matrix-core pair, one tile per 16-atom group g of the work order,
    // [g][S][K][4][16][4] (element (k, q, atom, i) = P[k][kMfmaRow[q][i]])
    float* Pbuf;
    // backward output: virial block partials
    double* vir;
};

struct Pair {
    float dx, dy, dz, r2;
    int q;     // neighbour (sorted index)
    int slot;  // where the entry's force goes: its LDS halo slot (LdsPos) or sorted index (GlobalPos)
};

template <int NB>
struct IntVec;
template <>
struct IntVec<2> {
    using T = int2;
    __device__ static void split(const int2& v, int* o) { o[0] = v.x, o[1] = v.y; }
};
template <>
struct IntVec<4> {
    using T = int4;
    __device__ static void split(const int4& v, int* o) { o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w; }
};

// Neighbour positions of list entries, in one of two places.  GlobalPos
// reads the sorted FP64 positions from HBM and forms D = (x_q - x_i) + n L in
// FP64.  LdsPos reads a workgroup's LDS copy of its cell block and one-cell
// halo, held as FP32 offsets from each atom's own cell origin: the entry's
// stencil offset (ox, oy, oz), stored as the bit fields ox+1, oy+1, oz+1 of
// its image word, names the halo slot (slot = centre's slot +
// (oz HY + oy) HX + ox; atom q of slot h sits at hoff[h] + q) and the cell
// offset, and D = (x_q - x_i) + o w with w the cell edge.  Both hand D to the
// caller in FP32 (the LDS form carries about 3e-7 A more rounding on |D| < 8 A).
struct GlobalPos {
    const double4* xs;
    double L0, L1, L2;
    double4 xi;
    __device__ double4 fetch(int q, int32_t, int& slot) const {
        slot = q;
        return xs[q];
    }
    __device__ float3 disp(const double4& xj, int32_t im) const {
        int nx, ny, nz;
        unpack_img(im, nx, ny, nz);
        return make_float3((float)((xj.x - xi.x) + (double)nx * L0), (float)((xj.y - xi.y) + (double)ny * L1),
                           (float)((xj.z - xi.z) + (double)nz * L2));
    }
};
struct LdsPos {
    const float* sx;
    const float* sy;
    const float* sz;
    const int32_t* hoff;
    int hp0;           // centre's halo slot minus (HX HY + HX + 1), the slot offset of the bit fields (0, 0, 0)
    int HX, HXY;       // halo cells along x, and per z layer
    float xi, yi, zi;  // centre atom from its cell origin, plus one cell edge
    float wx, wy, wz;  // cell edges
    __device__ float4 fetch(int q, int32_t im, int& slot) const {
        const int i = hoff[hp0 + img_sz(im) * HXY + img_sy(im) * HX + img_sx(im)] + q;
        slot = i;
        return make_float4(sx[i], sy[i], sz[i], 0.0f);
    }
    // (x_q - x_i) + (b - 1) w = x_q - (x_i + w) + b w for the field b = o + 1
    __device__ float3 disp(const float4& xj, int32_t im) const {
        return make_float3(fmaf((float)img_sx(im), wx, xj.x - xi), fmaf((float)img_sy(im), wy, xj.y - yi),
                           fmaf((float)img_sz(im), wz, xj.z - zi));
    }
};

// NB consecutive entries c0 .. c0+NB-1 (c0 a multiple of NB) of a list row of
// nb (>= 1) entries starting at `row` (16-byte aligned): one vector load each
// for indices and image words, then all position loads, so the loads overlap.
// Entries past the row end are replaced by the last valid entry (never a
// stale slot) and marked with r2 = +inf so that every consumer skips them.
template <int NB, class Pos>
__device__ __forceinline__ void load_pairs(const PathArgs& a, int64_t row, int c0, int nb, Pair (&pr)[NB],
                                           const Pos& pos) {
    int q[NB], im[NB];
    IntVec<NB>::split(*reinterpret_cast<const typename IntVec<NB>::T*>(a.nbr + row + c0), q);
    IntVec<NB>::split(*reinterpret_cast<const typename IntVec<NB>::T*>(a.img + row + c0), im);
#pragma unroll
    for (int j = 1; j < NB; ++j)
        if (c0 + j >= nb) {  // entry c0 < nb is always valid
            q[j] = q[0];
            im[j] = im[0];
        }
    int slot[NB];
    decltype(pos.fetch(0, 0, slot[0])) xj[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) xj[j] = pos.fetch(q[j], im[j], slot[j]);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const float3 d = pos.disp(xj[j], im[j]);
        pr[j].dx = d.x;
        pr[j].dy = d.y;
        pr[j].dz = d.z;
        pr[j].r2 = (c0 + j < nb) ? pr[j].dx * pr[j].dx + pr[j].dy * pr[j].dy + pr[j].dz * pr[j].dz
                                 : __builtin_inff();
        pr[j].q = q[j];
        pr[j].slot = slot[j];
    }
}

// The value of the neighbouring lane (lane ^ 1), by a DPP quad permutation
// [1, 0, 3, 2] (no LDS crossbar).
__device__ __forceinline__ float swap_pair(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// load_pairs for an atom whose list is walked by two adjacent lanes (its two
// radial chunks; both lanes see the same row): each lane fetches every other
// neighbour position and forms its displacement, and the two swap results, so
// the row's position gathers and FP64 geometry are done once per atom rather
// than once per lane.  The values are those of load_pairs bit for bit.
template <int NB, class Pos>
__device__ __forceinline__ void load_pairs_split2(const PathArgs& a, int64_t row, int c0, int nb, Pair (&pr)[NB],
                                                  const Pos& pos, int odd) {
    static_assert(NB % 2 == 0, "pairs are shared two at a time");
    int q[NB], im[NB];
    IntVec<NB>::split(*reinterpret_cast<const typename IntVec<NB>::T*>(a.nbr + row + c0), q);
    IntVec<NB>::split(*reinterpret_cast<const typename IntVec<NB>::T*>(a.img + row + c0), im);
#pragma unroll
    for (int j = 1; j < NB; ++j)
        if (c0 + j >= nb) {
            q[j] = q[0];
            im[j] = im[0];
        }
    int slot_unused;
    decltype(pos.fetch(0, 0, slot_unused)) xj[NB / 2];  // entries 2t + odd
#pragma unroll
    for (int t = 0; t < NB / 2; ++t)
        xj[t] = pos.fetch(odd ? q[2 * t + 1] : q[2 * t], odd ? im[2 * t + 1] : im[2 * t], slot_unused);
#pragma unroll
    for (int t = 0; t < NB / 2; ++t) {
        const float3 mine = pos.disp(xj[t], odd ? im[2 * t + 1] : im[2 * t]);
        const float3 other = make_float3(swap_pair(mine.x), swap_pair(mine.y), swap_pair(mine.z));
        const float3 d0 = odd ? other : mine, d1 = odd ? mine : other;
        pr[2 * t].dx = d0.x;
        pr[2 * t].dy = d0.y;
        pr[2 * t].dz = d0.z;
        pr[2 * t + 1].dx = d1.x;
        pr[2 * t + 1].dy = d1.y;
        pr[2 * t + 1].dz = d1.z;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        pr[j].r2 = (c0 + j < nb) ? pr[j].dx * pr[j].dx + pr[j].dy * pr[j].dy + pr[j].dz * pr[j].dz
                                 : __builtin_inff();
        pr[j].q = q[j];
        pr[j].slot = q[j];  // the descriptor has no force sink
    }
}

constexpr int kBatchFwd = 4;
constexpr int kBatchAdj = 2;

// A thread's KC x DR tile of P (its kept components) in the element-major
// buffer [S][K][DR][n]: element (k, r) of work slot w lives at
// ((b*K + k)*DR + r)*n + w, so for a fixed
// element the lanes of a wave (consecutive slots, two chunks) write and read
// whole contiguous cache lines.  P (2 GB at 1 M atoms) is written once and
// read once by the adjoint, far more than the L2 holds.  With at most two
// chunk lanes per atom every store instruction writes whole 128-byte lines,
// and those go out non-temporally (measured: less L2 pollution for the next
// kernel); with more chunks a store covers 32-byte pieces, which must merge in
// L2 (non-temporal stores were up to five times slower there).
template <int KC, int D, bool NT>
__device__ __forceinline__ void store_tile(float* dst, int64_t n, const float (&P)[KC][D]) {
#pragma unroll
    for (int q = 0; q < KC * D; ++q) {
        if constexpr (NT)
            __builtin_nontemporal_store(P[q / D][q % D], dst + (int64_t)q * n);
        else
            dst[(int64_t)q * n] = P[q / D][q % D];
    }
}

// Kept components (reduced index) of the matrix-core kernels' slices:
// entry n of slice q is kMfmaRow[q][n]; column n, (kMfmaRow[0..3][n]), is fold
// set n: the three kept components tied by the unit-norm identity to one
// dropped component, and one more.
__device__ constexpr int kMfmaRow[4][4] = {{0, 1, 2, 3}, {4, 9, 10, 11}, {7, 12, 14, 15}, {5, 6, 8, 13}};

// The same tile (M = 3) in the atom-major layout [n][S][K][4][4] read by the
// large-K matrix-core adjoint, one atom at a time: per radial function the
// four fold sets, each a float4 (kMfmaRow[0..3][g]), so that a lane loads its
// fold set with one instruction.
template <int KC, int D>
__device__ __forceinline__ void store_tile_am(float* dst, const float (&P)[KC][D]) {
    static_assert(D == 16, "the 16-component basis");
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
        for (int g = 0; g < 4; ++g)
            *reinterpret_cast<float4*>(dst + kk * 16 + 4 * g) =
                make_float4(P[kk][kMfmaRow[0][g]], P[kk][kMfmaRow[1][g]], P[kk][kMfmaRow[2][g]], P[kk][kMfmaRow[3][g]]);
}

template <int KC, int D>
__device__ __forceinline__ void load_tile(const float* src, int64_t n, float (&P)[KC][D]) {
#pragma unroll
    for (int q = 0; q < KC * D; ++q) P[q / D][q % D] = src[(int64_t)q * n];
}

// Gaussians exp(-eta_k (R - mu_k)^2) of a chunk of KC radial functions
// (mu, nef = -eta log2 e of the chunk).  On a uniform grid (a.rec) two
// exponentials and a multiplicative recurrence replace the KC exponentials:
// e_{k+1} = e_k r_k, r_k = exp2(rec_a (R - mu_k) + rec_b), r_{k+1} = r_k rec_c.
template <int KC>
__device__ __forceinline__ void gaussians_rec(const PathArgs& a, float R, const float* mu, const float* nef,
                                              float (&e)[KC]) {
    const float t0 = R - mu[0];
    float ek = __builtin_amdgcn_exp2f(nef[0] * t0 * t0);
    float rk = __builtin_amdgcn_exp2f(fmaf(a.rec_a, t0, a.rec_b));
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        e[kk] = ek;
        ek *= rk;
        rk *= a.rec_c;
    }
}
template <int KC>
__device__ __forceinline__ void gaussians_direct(float R, const float* mu, const float* nef, float (&e)[KC]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const float t = R - mu[kk];
        e[kk] = __builtin_amdgcn_exp2f(nef[kk] * t * t);
    }
}
template <int KC>
__device__ __forceinline__ void gaussians(const PathArgs& a, float R, const float* mu, const float* nef,
                                          float (&e)[KC]) {
    if (a.rec) gaussians_rec<KC>(a, R, mu, nef, e);
    else gaussians_direct<KC>(R, mu, nef, e);
}

// How the adjoint kernels evaluate the radial functions (a template
// parameter, so that each instantiation keeps only its own registers):
// directly, by the uniform-grid recurrence, or from the table.
constexpr int kRadDirect = 0, kRadRec = 1, kRadTab = 2;

// Chunk k0 .. k0+KC-1 of the tabulated radial functions at distance R (the
// caller has R < rc): interval j = floor(R / delta), clamped to the zero row
// tab_n, local t = R / delta - j, h = c0 + t(c1 + t(c2 + t c3)) and, with DH,
// h' = (c1 + t(2 c2 + 3 t c3)) / delta.  The KC coefficient quadruples of a
// thread are one contiguous 16*KC-byte run of the table.
template <int KC, bool DH>
__device__ __forceinline__ void tabulated(const PathArgs& a, float R, int k0, float (&h)[KC], float (&dh)[KC]) {
    const float x = R * a.tab_inv;
    const float jf = fminf(floorf(x), (float)a.tab_n);
    const float t = x - jf;
    const float4* row = a.tab + (int64_t)jf * a.K + k0;
    float4 c[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) c[kk] = row[kk];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        h[kk] = fmaf(t, fmaf(t, fmaf(t, c[kk].w, c[kk].z), c[kk].y), c[kk].x);
        if (DH) dh[kk] = fmaf(t, fmaf(3.0f * t, c[kk].w, 2.0f * c[kk].z), c[kk].y) * a.tab_inv;
    }
}

// P tile of one species for this thread's radial chunk.
template <int KC, int M, bool TAB, class Pos>
__device__ __forceinline__ void accumulate_P(const PathArgs& a, int64_t p, int b, int k0, const float* mu,
                                             const float* nef, float (&P)[KC][Moments<M>::DR], const Pos& pos) {
    constexpr int D = Moments<M>::DR;  // the kept components (reduced_monomials)
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
        for (int d = 0; d < D; ++d) P[kk][d] = 0.0f;
    const int nb = a.cnt[(int64_t)b * a.n + p];
    const int64_t base = (p * a.S + b) * a.cap;  // row of (atom, species)
    for (int c0 = 0; c0 < nb; c0 += kBatchFwd) {
      Pair prs[kBatchFwd];
      if (a.nch_log2 == 1)  // uniform: two chunk lanes per atom share the geometry
          load_pairs_split2<kBatchFwd>(a, base, c0, nb, prs, pos, (k0 / KC) & 1);
      else
          load_pairs<kBatchFwd>(a, base, c0, nb, prs, pos);
#pragma unroll
      for (int j = 0; j < kBatchFwd; ++j) {
        const Pair& pr = prs[j];
        if (pr.r2 >= a.rc2) continue;
        const float rinv = __builtin_amdgcn_rsqf(pr.r2);
        const float R = pr.r2 * rinv;
        const float ux = pr.dx * rinv, uy = pr.dy * rinv, uz = pr.dz * rinv;
        float Mv[D], hv[KC];
        reduced_monomials<M>(ux, uy, uz, Mv);
        if (TAB) {
            tabulated<KC, false>(a, R, k0, hv, hv);
        } else {
            const float fc = 0.5f * __builtin_amdgcn_cosf(R * a.half_inv_rc) + 0.5f;
            gaussians<KC>(a, R, mu, nef, hv);
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) hv[kk] *= fc;
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
            for (int d = 0; d < D; ++d) P[kk][d] = fmaf(hv[kk], Mv[d], P[kk][d]);
        }
      }
    }
}

// PL: where P goes (0 element-major, 1 element-major non-temporal, 2 atom-major).
template <int KC, int M, bool TAB, int PL>
__global__ void __launch_bounds__(256, KC <= 4 ? 3 : 2) k_descriptor(PathArgs a, int64_t nblocks) {
    constexpr int D = Moments<M>::D, DR = Moments<M>::DR;
    constexpr int GW = KC * (M + 1);  // features of one thread's chunk
    // Per wave: its atoms' feature segments of two species, so that G's rows
    // go out as consecutive floats (a lane-per-atom store would touch one
    // cache line per lane) and, with two species, as whole rows (a row
    // written one species at a time leaves a cache line half written in
    // between), and the atoms' sorted indices.
    __shared__ float sg[kBlock / 64][2 * 64 * GW + 64];  // rows padded to an odd stride (banks)
    __shared__ int32_t sp_row[kBlock / 64][64];
    const int64_t lb = xcd_block(nblocks);
    if (lb < 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = lb * blockDim.x + threadIdx.x;
    const int64_t w = t >> a.nch_log2;  // work slot
    const int ch = (int)(t & ((1 << a.nch_log2) - 1));
    const bool active = w < a.n;
    const int64_t p = active ? (a.wperm ? a.wperm[w] : w) : 0;
    if (ch == 0) sp_row[wv][lane >> a.nch_log2] = (int32_t)p;
    const int64_t wave_w0 = (lb * blockDim.x + (threadIdx.x & ~63)) >> a.nch_log2;
    const int KM = a.K * (M + 1);  // features of one species
    float mu[KC], nef[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        mu[kk] = a.mu[ch * KC + kk];
        nef[kk] = -a.eta[ch * KC + kk] * kLog2e;
    }
    const double4 Lp = a.boxes ? a.boxes[p] : make_double4(a.L[0], a.L[1], a.L[2], 0.0);
    const GlobalPos pos{a.xs, Lp.x, Lp.y, Lp.z, a.xs[p]};
    for (int b = 0; b < a.S; ++b) {
        const int b0 = b & ~1;                // species b0 and b0 + 1 are staged together
        const int nsp = min(2, a.S - b0);     // species in this pair
        const int RW = nsp * KM;              // staged floats per atom
        const int RWp = RW | 1;               // their LDS stride
        if (active) {
            float Pr[KC][DR], P[KC][D];
            accumulate_P<KC, M, TAB>(a, p, b, ch * KC, mu, nef, Pr, pos);
            if (a.Pbuf) {
                if constexpr (PL == 2)
                    store_tile_am<KC, DR>(a.Pbuf + (((int64_t)w * a.S + b) * a.K + ch * KC) * DR, Pr);
                else
                    store_tile<KC, DR, PL == 1>(a.Pbuf + ((int64_t)(b * a.K + ch * KC) * DR) * a.n + w, a.n, Pr);
            }
            expand_P<M, KC>(Pr, P);
            float* seg = &sg[wv][(lane >> a.nch_log2) * RWp + (b - b0) * KM + ch * GW];
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
                for (int m = 0; m <= M; ++m) {
                    float s = 0.0f;
#pragma unroll
                    for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) s += kMult[d] * P[kk][d] * P[kk][d];
                    // m = 0 has the single component d = 0: sqrt(S) = |P_k0| exactly
                    seg[kk * (M + 1) + m] = (m == 0) ? fabsf(P[kk][0]) : s;
                }
            }
        }
        if (b - b0 < nsp - 1) continue;  // uniform: the pair's second species is still to come
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the wave's (64 / chunks) atoms x RW features, 64 consecutive floats per
        // store: feature e of atom al is staged at al * RWp + e
        int al = lane / RW, e = lane - al * RW;
        for (int it = 0; it < nsp * GW; ++it) {
            if (wave_w0 + al < a.n) {
                const int64_t gi = (int64_t)sp_row[wv][al] * a.F + b0 * KM + e;
                const float gx = sg[wv][al * RWp + e];
                if (a.Gb)
                    a.Gb[gi] = __builtin_bit_cast(uint16_t, (__bf16)gx);
                else
                    a.G[gi] = gx;
            }
            e += 64;
            while (e >= RW) {
                e -= RW;
                ++al;
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---- adjoint ---------------------------------------------------------------
//
// Force sums.  Each pair's g is added to the neighbour's force (F_j -= g) by
// an atomic add, first into the workgroup's LDS accumulators and then into
// the global ones.  The adds are made on 64-bit fixed-point integers with 32
// fractional bits: integer addition is associative, so the result does not
// depend on the order in which the atomics land and the forces are the same
// bit for bit on every run (float atomics would round in arrival order).
// A contribution g is split as g = hi + fr with hi = floor(g) (an integer,
// exact in FP32 for |g| < 2^31) and fr in [0, 1) (exact); fr 2^32 is exact
// too and converts to the low word (truncating only bits below 2^-32), hi to
// the high word, which together are the two's-complement integer g 2^32.
__device__ __forceinline__ unsigned long long to_fixed(float g) {
    const float hi = floorf(g);
    const unsigned lo = (unsigned)((g - hi) * 4294967296.0f);
    return ((unsigned long long)(unsigned)(int)hi << 32) | lo;
}

// P' = 2 T sigma' P in place for one species' KC x D tile (sigma' = dE/dS
// from dE/dG): for m = 0, G = sqrt(P_k0^2) = |P_k0|, so P'_k0 = G' sign(P_k0)
// (0 where P_k0 = 0; no reciprocal square root of a possibly denormal S).
template <int KC, int M>
__device__ __forceinline__ void tile_adjoint(const float* dGp, float (&P)[KC][Moments<M>::D]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
        for (int m = 0; m <= M; ++m) {
            const float gbar = dGp[kk * (M + 1) + m];
            if (m == 0) {
                const float pk = P[kk][0];
                P[kk][0] = pk > 0.0f ? gbar : (pk < 0.0f ? -gbar : 0.0f);
            } else {
#pragma unroll
                for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) P[kk][d] *= 2.0f * kMult[d] * gbar;
            }
        }
    }
}

// This thread's P' tile of species b in the kept basis: the stored kept
// components of P, expanded, turned into P' and folded back.
template <int KC, int M>
__device__ __forceinline__ void adjoint_tile(const PathArgs& a, int64_t p, int64_t w, int b, int ch,
                                             float (&Pr)[KC][Moments<M>::DR]) {
    constexpr int D = Moments<M>::D, DR = Moments<M>::DR;
    float P[KC][D];
    load_tile<KC, DR>(a.Pbuf + ((int64_t)(b * a.K + ch * KC) * DR) * a.n + w, a.n, Pr);
    expand_P<M, KC>(Pr, P);
    tile_adjoint<KC, M>(a.dG + p * a.F + (b * a.K + ch * KC) * (M + 1), P);
    fold_Pbar<M, KC>(P, Pr);
}

// This chunk's share of g = dE/dD for one pair within the cutoff:
// U_k = sum_d P'_kd M_d, V_d = sum_k P'_kd h_k,
// g = (sum_k U_k h'_k) u + (1/R)(sum_d V_d grad_u M_d - u sum_d ord(d) V_d M_d).
template <int KC, int M, int RAD>
__device__ __forceinline__ void pair_grad(const PathArgs& a, float dx, float dy, float dz, float r2, int k0,
                                          const float* mu, const float* nef, const float* m2eta,
                                          const float (&P)[KC][Moments<M>::DR], float& gx, float& gy, float& gz) {
    constexpr int D = Moments<M>::DR;  // P' folded onto the kept basis (fold_Pbar)
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float R = r2 * rinv;
    const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
    float Mv[D];
    reduced_monomials<M>(ux, uy, uz, Mv);
    float V[D];
#pragma unroll
    for (int d = 0; d < D; ++d) V[d] = 0.0f;
    if constexpr (RAD == kRadRec) {
        // Uniform grid (mu_k = mu_0 + k Delta, one eta): with e_k the bare
        // Gaussians, h_k = e_k f_c and h'_k = e_k (-2 eta (t0 - k Delta) f_c + f_c'),
        // t0 = R - mu_0, so sum_k U_k h'_k = -2 eta f_c (t0 S0 - Delta S1) + f_c' S0
        // with S0 = sum_k U_k e_k and S1 = sum_k k U_k e_k, and f_c, being common
        // to every V_d, factors out of the moment adjoint.
        const float ang = R * a.half_inv_rc;
        const float fc = 0.5f * __builtin_amdgcn_cosf(ang) + 0.5f;
        const float dfc = -0.5f * a.pi_over_rc * __builtin_amdgcn_sinf(ang);
        float e[KC];
        gaussians_rec<KC>(a, R, mu, nef, e);
        float S0 = 0.0f, S1 = 0.0f;
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            float U = 0.0f;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                U = fmaf(P[kk][d], Mv[d], U);
                V[d] = fmaf(P[kk][d], e[kk], V[d]);
            }
            const float Ue = U * e[kk];
            S0 += Ue;
            S1 = fmaf((float)kk, Ue, S1);
        }
        const float t0 = R - mu[0];
        const float s1 = fmaf(a.rec_m2eta * fc, fmaf(-a.rec_delta, S1, t0 * S0), dfc * S0);
        float Ax, Ay, Az, B;
        reduced_moment_adjoint<M>(ux, uy, uz, V, Mv, Ax, Ay, Az, B);
        const float rf = rinv * fc;
        gx = s1 * ux + rf * (Ax - ux * B);
        gy = s1 * uy + rf * (Ay - uy * B);
        gz = s1 * uz + rf * (Az - uz * B);
        return;
    }
    float s1 = 0.0f, hv[KC], dhv[KC];
    if constexpr (RAD == kRadTab) {
        tabulated<KC, true>(a, R, k0, hv, dhv);
    } else {
        const float ang = R * a.half_inv_rc;
        const float fc = 0.5f * __builtin_amdgcn_cosf(ang) + 0.5f;
        const float dfc = -0.5f * a.pi_over_rc * __builtin_amdgcn_sinf(ang);
        gaussians_direct<KC>(R, mu, nef, hv);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const float e = hv[kk];
            hv[kk] = e * fc;
            dhv[kk] = e * fmaf(m2eta[kk] * (R - mu[kk]), fc, dfc);
        }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const float h = hv[kk];
        const float dh = dhv[kk];
        float U = 0.0f;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            U = fmaf(P[kk][d], Mv[d], U);
            V[d] = fmaf(P[kk][d], h, V[d]);
        }
        s1 = fmaf(U, dh, s1);
    }
    float Ax, Ay, Az, B;
    reduced_moment_adjoint<M>(ux, uy, uz, V, Mv, Ax, Ay, Az, B);
    gx = s1 * ux + rinv * (Ax - ux * B);
    gy = s1 * uy + rinv * (Ay - uy * B);
    gz = s1 * uz + rinv * (Az - uz * B);
}

// Virial of one pair: w6 -= D (x) g, off-diagonals symmetrised.
__device__ __forceinline__ void virial_add(float (&w6)[6], float dx, float dy, float dz, float gx, float gy, float gz) {
    w6[0] -= dx * gx;
    w6[1] -= dy * gy;
    w6[2] -= dz * gz;
    w6[3] -= 0.5f * (dx * gy + dy * gx);
    w6[4] -= 0.5f * (dx * gz + dz * gx);
    w6[5] -= 0.5f * (dy * gz + dz * gy);
}

// Radial parameters of this thread's chunk k0 .. k0+KC-1.
template <int KC>
__device__ __forceinline__ void chunk_params(const PathArgs& a, int k0, float (&mu)[KC], float (&nef)[KC],
                                             float (&m2eta)[KC]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        mu[kk] = a.mu[k0 + kk];
        nef[kk] = -a.eta[k0 + kk] * kLog2e;
        m2eta[kk] = -2.0f * a.eta[k0 + kk];
    }
}

// Per-atom adjoint for one (atom, radial chunk) thread with any number nch of
// chunk lanes per atom: P' from dE/dG, then for every pair U, V and g = dE/dD
// (summed over the atom's chunk lanes by shuffles).  The chunk-0 lane hands
// each pair's g to sink(slot, gx, gy, gz) (slot = where the neighbour's force
// accumulates: Pair::slot), accumulates the atom's own force sum in Fo and
// the virial: per species row in FP32 (like an atomic energy), added to the
// FP64 per-thread sums Wd after each row.
template <int KC, int M, int RAD, class Pos, class Sink>
__device__ __forceinline__ void adjoint_atom(const PathArgs& a, int64_t p, int64_t w, int ch, int nch,
                                             double (&Wd)[6], float (&Fo)[3], const Pos& pos, Sink&& sink) {
    constexpr int DR = Moments<M>::DR;
    float mu[KC], nef[KC], m2eta[KC];
    chunk_params<KC>(a, ch * KC, mu, nef, m2eta);
    for (int b = 0; b < a.S; ++b) {
        float P[KC][DR];
        adjoint_tile<KC, M>(a, p, w, b, ch, P);
        const int nb = a.cnt[(int64_t)b * a.n + p];
        const int64_t base = (p * a.S + b) * a.cap;  // row of (atom, species)
        float w6[6] = {0, 0, 0, 0, 0, 0};
        for (int c0 = 0; c0 < nb; c0 += kBatchAdj) {
            Pair prs[kBatchAdj];
            load_pairs<kBatchAdj>(a, base, c0, nb, prs, pos);
#pragma unroll
            for (int j = 0; j < kBatchAdj; ++j) {
                const Pair& pr = prs[j];
                if (pr.r2 >= a.rc2) continue;  // skin entries and padding carry no force
                float gx, gy, gz;
                pair_grad<KC, M, RAD>(a, pr.dx, pr.dy, pr.dz, pr.r2, ch * KC, mu, nef, m2eta, P, gx, gy, gz);
                for (int off = 1; off < nch; off <<= 1) {
                    gx += __shfl_xor(gx, off);
                    gy += __shfl_xor(gy, off);
                    gz += __shfl_xor(gz, off);
                }
                if (ch == 0) {
                    Fo[0] += gx;
                    Fo[1] += gy;
                    Fo[2] += gz;
                    sink(pr.slot, gx, gy, gz);
                    virial_add(w6, pr.dx, pr.dy, pr.dz, gx, gy, gz);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) Wd[j] += (double)w6[j];
    }
}

// The same for exactly two chunk lanes per atom (K = 2 KC), the lanes t and
// t ^ 1 of a wave.  The pairs go two at a time, and the work of a pair that
// does not depend on the chunk is split between the lanes: lane `odd` fetches
// entry c0 + odd (its halo slot and position) and forms its displacement, and
// the lanes swap displacements by a DPP lane permutation; both lanes then run
// their chunk's share of both pairs, sum the two shares by the same
// permutation, and lane `odd` adds pair c0 + odd to the force sums and the
// virial.  Every value is the one the generic form computes; the two lanes of
// an atom always run together (same row, same r2 for each pair), so the lane
// permutations always find their partner active.
template <int KC, int M, int RAD, class Sink>
__device__ __forceinline__ void adjoint_atom_pair2(const PathArgs& a, int64_t p, int64_t w, int ch, double (&Wd)[6],
                                                   float (&Fo)[3], const LdsPos& pos, Sink&& sink) {
    constexpr int DR = Moments<M>::DR;
    const int odd = ch & 1;
    float mu[KC], nef[KC], m2eta[KC];
    chunk_params<KC>(a, ch * KC, mu, nef, m2eta);
    for (int b = 0; b < a.S; ++b) {
        float P[KC][DR];
        adjoint_tile<KC, M>(a, p, w, b, ch, P);
        const int nb = a.cnt[(int64_t)b * a.n + p];
        const int64_t base = (p * a.S + b) * a.cap;  // row of (atom, species), 16-byte aligned
        float w6[6] = {0, 0, 0, 0, 0, 0};
        for (int c0 = 0; c0 < nb; c0 += 2) {
            const int2 qv = *reinterpret_cast<const int2*>(a.nbr + base + c0);
            const int2 iv = *reinterpret_cast<const int2*>(a.img + base + c0);
            const bool v1 = c0 + 1 < nb;  // past the row's end entry c0 + 1 repeats entry c0, marked out of range
            const int q = (odd && v1) ? qv.y : qv.x;
            const int im = (odd && v1) ? iv.y : iv.x;
            int slot;
            const float4 xj = pos.fetch(q, im, slot);
            const float3 dm = pos.disp(xj, im);
            const float ox = swap_pair(dm.x), oy = swap_pair(dm.y), oz = swap_pair(dm.z);
            const float d0x = odd ? ox : dm.x, d0y = odd ? oy : dm.y, d0z = odd ? oz : dm.z;
            const float d1x = odd ? dm.x : ox, d1y = odd ? dm.y : oy, d1z = odd ? dm.z : oz;
            const float r20 = d0x * d0x + d0y * d0y + d0z * d0z;
            const float r21 = v1 ? d1x * d1x + d1y * d1y + d1z * d1z : __builtin_inff();
            float g0x = 0.0f, g0y = 0.0f, g0z = 0.0f, g1x = 0.0f, g1y = 0.0f, g1z = 0.0f;
            if (r20 < a.rc2)  // skin entries and padding carry no force
                pair_grad<KC, M, RAD>(a, d0x, d0y, d0z, r20, ch * KC, mu, nef, m2eta, P, g0x, g0y, g0z);
            if (r21 < a.rc2)
                pair_grad<KC, M, RAD>(a, d1x, d1y, d1z, r21, ch * KC, mu, nef, m2eta, P, g1x, g1y, g1z);
            g0x += swap_pair(g0x);
            g0y += swap_pair(g0y);
            g0z += swap_pair(g0z);
            g1x += swap_pair(g1x);
            g1y += swap_pair(g1y);
            g1z += swap_pair(g1z);
            if ((odd ? r21 : r20) < a.rc2) {
                const float gx = odd ? g1x : g0x, gy = odd ? g1y : g0y, gz = odd ? g1z : g0z;
                Fo[0] += gx;
                Fo[1] += gy;
                Fo[2] += gz;
                sink(slot, gx, gy, gz);
                virial_add(w6, dm.x, dm.y, dm.z, gx, gy, gz);
            }
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) Wd[j] += (double)w6[j];
    }
}

struct CompD {
    double s, c;
};
__device__ __forceinline__ CompD comp_merge_d(CompD a, CompD b) {
    const double t = a.s + b.s;
    if (fabs(a.s) >= fabs(b.s)) a.c += (a.s - t) + b.s;
    else a.c += (b.s - t) + a.s;
    a.s = t;
    a.c += b.c;
    return a;
}

// Block reduction of the per-thread FP64 virial sums (256 threads) into
// out[12] = six Neumaier-compensated sums (value, compensation), in a fixed
// order: a butterfly inside each wave, then the four waves in turn.
__device__ __forceinline__ void block_virial(const double (&Wd)[6], double (*red)[kBlock / 64][2], double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        CompD v{Wd[j], 0.0};
        for (int off = 32; off > 0; off >>= 1) {
            const CompD o{__shfl_xor(v.s, off), __shfl_xor(v.c, off)};
            v = (lane & off) ? comp_merge_d(o, v) : comp_merge_d(v, o);
        }
        if (lane == 0) {
            red[j][wv][0] = v.s;
            red[j][wv][1] = v.c;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        CompD r{0.0, 0.0};
        for (int w = 0; w < kBlock / 64; ++w) r = comp_merge_d(r, CompD{red[threadIdx.x][w][0], red[threadIdx.x][w][1]});
        out[2 * threadIdx.x] = r.s;
        out[2 * threadIdx.x + 1] = r.c;
    }
}

// Adjoint with the force scatter done by device-scope atomics: used only when
// the stencil is wider than 3x3x3 (a box edge shorter than two list cutoffs).
template <int KC, int M, int RAD>
__global__ void __launch_bounds__(256) k_adjoint_atomic(PathArgs a, unsigned long long* F) {
    __shared__ double red[6][kBlock / 64][2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = t >> a.nch_log2;
    const int nch = 1 << a.nch_log2;
    const int ch = (int)(t & (nch - 1));
    double Wd[6] = {0, 0, 0, 0, 0, 0};
    if (w < a.n) {
        const int64_t p = a.wperm ? a.wperm[w] : w;
        float Fo[3] = {0.0f, 0.0f, 0.0f};
        const double4 Lp = a.boxes ? a.boxes[p] : make_double4(a.L[0], a.L[1], a.L[2], 0.0);
        adjoint_atom<KC, M, RAD>(a, p, w, ch, nch, Wd, Fo, GlobalPos{a.xs, Lp.x, Lp.y, Lp.z, a.xs[p]},
                                 [&](int q, float gx, float gy, float gz) {
            atomicAdd(&F[3 * (int64_t)q + 0], to_fixed(-gx));
            atomicAdd(&F[3 * (int64_t)q + 1], to_fixed(-gy));
            atomicAdd(&F[3 * (int64_t)q + 2], to_fixed(-gz));
        });
        if (ch == 0) {
            atomicAdd(&F[3 * p + 0], to_fixed(Fo[0]));
            atomicAdd(&F[3 * p + 1], to_fixed(Fo[1]));
            atomicAdd(&F[3 * p + 2], to_fixed(Fo[2]));
        }
    }
    block_virial(Wd, red, a.vir + (int64_t)blockIdx.x * kVirDoubles);
}

struct BlockGeom {
    int nc[3];   // cells per dimension
    int B[3];    // cells per block and dimension
    int nb[3];   // blocks per dimension
    int hmax;    // capacity of the LDS force accumulators (atoms)
    const int32_t* cellstart;
    unsigned long long* F;  // fixed-point forces [n][3]
    const int32_t* wbase;  // [blocks + 1] first work slot of each block
    // [blocks + 1] first 16-atom group of each block in the matrix-core P
    // layout (a block of c atoms takes ceil(c / 16) groups)
    const int32_t* gbase;
    const int32_t* wperm;  // work slot -> sorted atom
    const uint8_t* wcell;  // work slot -> cell inside its block
};

constexpr int kMaxHaloCells = 216;    // (4 + 2)^3
constexpr int kMaxBlockCells = 64;    // 4^3

__device__ __forceinline__ int wrap_cell(int c, int nc) {
    c %= nc;
    return c < 0 ? c + nc : c;
}

// Exclusive prefix sum of one value per thread over the 256 threads of a block.
__device__ __forceinline__ void scan256(int v, int32_t* out, int32_t* wtmp) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wtmp[wv] = x;
    __syncthreads();
    int pre = 0;
    for (int w = 0; w < wv; ++w) pre += wtmp[w];
    out[t] = pre + x - v;
    if (t == 255) out[256] = pre + x;
    __syncthreads();
}

// Halo slots of block lb: h_first[h] = first sorted atom of slot h's cell,
// h_base = exclusive scan of the slot counts (h_base[nh] = halo atoms),
// hoff[h] = h_base[h] - h_first[h].  Ends with a barrier.
__device__ __forceinline__ void halo_slots(const BlockGeom& bg, int64_t lb, int32_t* h_first, int32_t* h_base,
                                           int32_t* hoff, int32_t* wtmp, int& x0, int& y0, int& z0) {
    const int t = threadIdx.x;
    const int bx = (int)(lb % bg.nb[0]), by = (int)((lb / bg.nb[0]) % bg.nb[1]), bz = (int)(lb / (bg.nb[0] * bg.nb[1]));
    x0 = bx * bg.B[0];
    y0 = by * bg.B[1];
    z0 = bz * bg.B[2];
    const int HX = bg.B[0] + 2, HY = bg.B[1] + 2, HZ = bg.B[2] + 2;
    const int nh = HX * HY * HZ;
    int hcount = 0;
    if (t < nh) {
        const int hx = t % HX, hy = (t / HX) % HY, hz = t / (HX * HY);
        const int gc = (wrap_cell(z0 - 1 + hz, bg.nc[2]) * bg.nc[1] + wrap_cell(y0 - 1 + hy, bg.nc[1])) * bg.nc[0] +
                       wrap_cell(x0 - 1 + hx, bg.nc[0]);
        h_first[t] = bg.cellstart[gc];
        hcount = bg.cellstart[gc + 1] - h_first[t];
    }
    scan256(hcount, h_base, wtmp);
    if (t < nh) hoff[t] = h_base[t] - h_first[t];
    __syncthreads();
}

// Positions of the halo atoms into sx, sy, sz (slot order) as FP32 offsets
// from the origin of the atom's own cell (cell c spans [c w, (c+1) w)).
// Ends with a barrier.
__device__ __forceinline__ void halo_positions(const BlockGeom& bg, const PathArgs& a, int x0, int y0, int z0,
                                               const int32_t* h_first, const int32_t* h_base, float* sx, float* sy,
                                               float* sz) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int HX = bg.B[0] + 2, HY = bg.B[1] + 2, HZ = bg.B[2] + 2;
    for (int hc = wv; hc < HX * HY * HZ; hc += kBlock / 64) {
        const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
        const double ox = (double)wrap_cell(x0 - 1 + hx, bg.nc[0]) * (a.L[0] / bg.nc[0]);
        const double oy = (double)wrap_cell(y0 - 1 + hy, bg.nc[1]) * (a.L[1] / bg.nc[1]);
        const double oz = (double)wrap_cell(z0 - 1 + hz, bg.nc[2]) * (a.L[2] / bg.nc[2]);
        const int lo = h_base[hc], cnt = h_base[hc + 1] - lo;
        for (int k = lane; k < cnt; k += 64) {
            const double4 x = a.xs[h_first[hc] + k];
            sx[lo + k] = (float)(x.x - ox);
            sy[lo + k] = (float)(x.y - oy);
            sz[lo + k] = (float)(x.z - oz);
        }
    }
    __syncthreads();
}

// Adjoint over one block of B0 x B1 x B2 cells (ScatterSum, Sec. III.A, done
// in two levels like the paper's partial-then-global reduction).  The
// workgroup first copies the positions of the block and its one-cell halo
// into LDS (FP32 offsets from each atom's cell origin), and its pair loops
// read neighbour positions there (LdsPos) instead of gathering them from HBM.
// The forces on the block's atoms and on its halo accumulate in LDS with LDS
// atomics (fixed point, so that the sums do not depend on their order),
// located through the stencil offset each list entry recorded; the block then
// adds its accumulators to F with device atomics, one range per halo cell.
// PAIR2: two chunk lanes per atom (adjoint_atom_pair2).
template <int KC, int M, int RAD, bool PAIR2>
__global__ void __launch_bounds__(256) k_adjoint_blocked(PathArgs a, BlockGeom bg) {
    // [3][hmax] halo positions (floats), then [3][hmax] fixed-point force accumulators
    extern __shared__ __attribute__((aligned(8))) unsigned char lds_dyn[];
    __shared__ int32_t h_base[257], h_first[kMaxHaloCells], hoff[kMaxHaloCells];
    __shared__ int32_t wtmp[kBlock / 64];
    __shared__ double red[6][kBlock / 64][2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int blk = blockIdx.x;
    int x0, y0, z0;
    halo_slots(bg, blk, h_first, h_base, hoff, wtmp, x0, y0, z0);
    const int HX = bg.B[0] + 2, HY = bg.B[1] + 2, HZ = bg.B[2] + 2;
    const int nh = HX * HY * HZ;
    const int hpos = (3 * bg.hmax + 1) & ~1;  // floats of the positions, rounded to 8 bytes
    float* sx = reinterpret_cast<float*>(lds_dyn);
    float* sy = sx + bg.hmax;
    float* sz = sx + 2 * bg.hmax;
    unsigned long long* sF = reinterpret_cast<unsigned long long*>(sx + hpos);
    const int htot = h_base[nh];
    for (int i = t; i < htot; i += kBlock) {
        sF[i] = 0ull;
        sF[bg.hmax + i] = 0ull;
        sF[2 * bg.hmax + i] = 0ull;
    }
    halo_positions(bg, a, x0, y0, z0, h_first, h_base, sx, sy, sz);  // ends with a barrier
    const float cw[3] = {(float)(a.L[0] / bg.nc[0]), (float)(a.L[1] / bg.nc[1]), (float)(a.L[2] / bg.nc[2])};
    // the block's atoms are work slots wbase[blk] .. wbase[blk+1], ordered by row length
    const int nch = 1 << a.nch_log2;
    const int64_t w0 = bg.wbase[blk];
    const int items = (int)(bg.wbase[blk + 1] - w0) << a.nch_log2;
    double Wd[6] = {0, 0, 0, 0, 0, 0};
    auto sink = [&](int idx, float gx, float gy, float gz) {  // idx: the neighbour's halo slot
        atomicAdd(&sF[idx], to_fixed(-gx));
        atomicAdd(&sF[bg.hmax + idx], to_fixed(-gy));
        atomicAdd(&sF[2 * bg.hmax + idx], to_fixed(-gz));
    };
    for (int item = t; item < ((items + kBlock - 1) / kBlock) * kBlock; item += kBlock) {
        if (item >= items) continue;
        const int ch = item & (nch - 1);
        const int64_t w = w0 + (item >> a.nch_log2);
        const int64_t p = bg.wperm[w];
        const int ic = bg.wcell[w];
        const int ix = ic % bg.B[0] + 1, iy = (ic / bg.B[0]) % bg.B[1] + 1, iz = ic / (bg.B[0] * bg.B[1]) + 1;
        const int hp = (iz * HY + iy) * HX + ix;
        const int ip = hoff[hp] + (int)p;
        const LdsPos pos{sx, sy, sz, hoff, hp - (HX * HY + HX + 1), HX, HX * HY,
                         sx[ip] + cw[0], sy[ip] + cw[1], sz[ip] + cw[2], cw[0], cw[1], cw[2]};
        float Fo[3] = {0.0f, 0.0f, 0.0f};
        if constexpr (PAIR2) {
            adjoint_atom_pair2<KC, M, RAD>(a, p, w, ch, Wd, Fo, pos, sink);
            atomicAdd(&sF[ip], to_fixed(Fo[0]));
            atomicAdd(&sF[bg.hmax + ip], to_fixed(Fo[1]));
            atomicAdd(&sF[2 * bg.hmax + ip], to_fixed(Fo[2]));
        } else {
            adjoint_atom<KC, M, RAD>(a, p, w, ch, nch, Wd, Fo, pos, sink);
            if (ch == 0) {
                atomicAdd(&sF[ip], to_fixed(Fo[0]));
                atomicAdd(&sF[bg.hmax + ip], to_fixed(Fo[1]));
                atomicAdd(&sF[2 * bg.hmax + ip], to_fixed(Fo[2]));
            }
        }
    }
    __syncthreads();
    for (int hc = wv; hc < nh; hc += kBlock / 64) {
        const int lo = h_base[hc], cnt = h_base[hc + 1] - lo;
        for (int k = lane; k < cnt; k += 64) {
            const int64_t q = h_first[hc] + k;
            const unsigned long long fx = sF[lo + k], fy = sF[bg.hmax + lo + k], fz = sF[2 * bg.hmax + lo + k];
            if (fx) atomicAdd(&bg.F[3 * q + 0], fx);
            if (fy) atomicAdd(&bg.F[3 * q + 1], fy);
            if (fz) atomicAdd(&bg.F[3 * q + 2], fz);
        }
    }
    block_virial(Wd, red, a.vir + (int64_t)blockIdx.x * kVirDoubles);
}

// ---- adjoint on the matrix cores (M = 3, K a multiple of 4) ---------------
//
// For one (atom, neighbour species) the two contractions of the adjoint are
// small dense products over the radial index k, for every pair c:
//   V1_d(c) = sum_k P'_kd B1_k(c),   V2_d(c) = sum_k P'_kd B2_k(c),
// with (B1, B2) = (h_k, h'_k), or on a uniform grid (e_k, k e_k) for the bare
// Gaussians e_k (the fold of pair_grad).  The rest of a pair's g needs only
// these: sum_k U_k h'_k = sum_d M_d V2_d (or the fold's S0 = M.V1, S1 = M.V2)
// and A = sum_d V1_d grad_u M_d.  v_mfma_f32_4x4x1f32 makes 16 independent
// 4x4 outer-product updates per instruction: block i of the wave (lanes
// 4i .. 4i+3) is one atom; lane 4i+n holds pair n of the atom's current
// four; the A operand (one value per lane) is a 4-entry slice of the atom's
// P' column k, the B operand the lane's own B_k; the 4x4 result keeps column
// n in lane 4i+n.  After K accumulation steps on four slices every lane holds
// all 16 entries of V1 and V2 for its own pair, and forms its pair's g alone.
//
// Lane n of a block supplies P' entries of the kept basis in the slices
// (q = 0..3) {n, rb, rc, rf}: with n = 0: (1, xx, yy, xy), 1: (x, xxx, xyy, xz),
// 2: (y, xxy, yyy, yz), 3: (z, xxz, yyz, xyz).  Each lane's first three are
// exactly the kept components that the unit-norm identity ties to one
// dropped component (zz, xzz, yzz, zzz), so the fold of P' onto the kept
// basis stays inside the lane, and a lane computes its P' entries from its
// own four P components and dE/dG alone.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));

// Image word of the centre atom's own cell (stencil offset 0, 0, 0).
constexpr int32_t kCentreWord = (int32_t)(0x15u << 24);


template <int KQ, int RAD>
__global__ void __launch_bounds__(256, 2) k_adjoint_mfma(PathArgs a, BlockGeom bg) {
    constexpr int K = 4 * KQ, DR = Moments<3>::DR;
    constexpr bool KA = RAD == kRadRec && KQ <= 3;  // k P' as the second product's A operand
    extern __shared__ __attribute__((aligned(8))) unsigned char lds_dyn[];
    __shared__ int32_t h_base[257], h_first[kMaxHaloCells], hoff[kMaxHaloCells];
    __shared__ int32_t wtmp[kBlock / 64];
    __shared__ double red[6][kBlock / 64][2];
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int quad = lane >> 2, j = lane & 3;
    const int blk = blockIdx.x;
    int x0, y0, z0;
    halo_slots(bg, blk, h_first, h_base, hoff, wtmp, x0, y0, z0);
    const int HX = bg.B[0] + 2, HY = bg.B[1] + 2, HZ = bg.B[2] + 2;
    const int nh = HX * HY * HZ;
    const int hpos = (3 * bg.hmax + 1) & ~1;
    float* sx = reinterpret_cast<float*>(lds_dyn);
    float* sy = sx + bg.hmax;
    float* sz = sx + 2 * bg.hmax;
    unsigned long long* sF = reinterpret_cast<unsigned long long*>(sx + hpos);
    const int htot = h_base[nh];
    for (int i = t; i < htot; i += kBlock) {
        sF[i] = 0ull;
        sF[bg.hmax + i] = 0ull;
        sF[2 * bg.hmax + i] = 0ull;
    }
    halo_positions(bg, a, x0, y0, z0, h_first, h_base, sx, sy, sz);  // ends with a barrier
    const float cw[3] = {(float)(a.L[0] / bg.nc[0]), (float)(a.L[1] / bg.nc[1]), (float)(a.L[2] / bg.nc[2])};
    auto sink = [&](int idx, float gx, float gy, float gz) {
        atomicAdd(&sF[idx], to_fixed(-gx));
        atomicAdd(&sF[bg.hmax + idx], to_fixed(-gy));
        atomicAdd(&sF[2 * bg.hmax + idx], to_fixed(-gz));
    };
    // 2 x the multiplicities of this lane's kept components kMfmaRow[q][j] and
    // of its dropped one (full T_dm row order: xx 1, xy 2, yy 1, zz 1; x 1,
    // xz 2, xxx 1, xyy 3, xzz 3; y 1, yz 2, xxy 3, yyy 1, yzz 3; z 1, xxz 3,
    // yyz 3, xyz 6, zzz 1)
    const float c2b = j <= 1 ? 2.0f : 6.0f;
    const float c2c = (j & 1) ? 6.0f : 2.0f;
    const float c2f = j == 3 ? 12.0f : 4.0f;
    const float c2d = (j == 0 || j == 3) ? 2.0f : 6.0f;
    const float sel0 = j == 0 ? 1.0f : 0.0f, sel1 = 1.0f - sel0, sel3 = j == 3 ? 1.0f : 0.0f, sel3c = 1.0f - sel3;
    float mu0 = 0.0f, nef0 = 0.0f;
    if constexpr (RAD == kRadRec) {
        mu0 = a.mu[0];
        nef0 = -a.eta[0] * kLog2e;
    }
    const int64_t w0 = bg.wbase[blk];
    const int natoms = (int)(bg.wbase[blk + 1] - w0);
    double Wd[6] = {0, 0, 0, 0, 0, 0};
    // each wave takes 16 atoms at a time (one per block of four lanes)
    for (int base = wv * 16; base < natoms; base += kBlock / 4) {
        const int ia = base + quad;
        const bool aval = ia < natoms;
        const int64_t w = w0 + (aval ? ia : natoms - 1);
        const int64_t g = bg.gbase[blk] + base / 16;  // the 16-atom group of P
        const int64_t p = bg.wperm[w];
        const int ic = bg.wcell[w];
        const int ix = ic % bg.B[0] + 1, iy = (ic / bg.B[0]) % bg.B[1] + 1, iz = ic / (bg.B[0] * bg.B[1]) + 1;
        const int hp = (iz * HY + iy) * HX + ix;
        const int ip = hoff[hp] + (int)p;
        const LdsPos pos{sx, sy, sz, hoff, hp - (HX * HY + HX + 1), HX, HX * HY,
                         sx[ip] + cw[0], sy[ip] + cw[1], sz[ip] + cw[2], cw[0], cw[1], cw[2]};
        float Fo[3] = {0.0f, 0.0f, 0.0f};
        for (int b = 0; b < a.S; ++b) {
            // this lane's slices of P' (= 2 T sigma' P, folded onto the kept basis)
            float Ap[K][4];
            // P in the group layout: element (k, q, atom, i) of the group's
            // species-b tile is P[k][kMfmaRow[q][i]]; this lane takes i = j
            const float* Pb = a.Pbuf + ((int64_t)g * a.S + b) * (K * 256) + quad * 4 + j;
            const float4* g4 = reinterpret_cast<const float4*>(a.dG + p * a.F + (int64_t)b * K * 4);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float* Pk = Pb + k * 256;
                const float pa = Pk[0], pb = Pk[64], pc = Pk[128], pf = Pk[192];
                const float4 g = g4[k];
                // the lane's orders picked arithmetically (0/1 weights), so that
                // every lane loads the whole dE/dG quadruple with one instruction
                const float ga = fmaf(sel0, g.x, sel1 * g.y), gbc = fmaf(sel0, g.z, sel1 * g.w),
                            gf = fmaf(sel3, g.w, sel3c * g.z);
                // the dropped component (zz, xzz, yzz or zzz) = pa - pb - pc
                const float pd = c2d * gbc * (pa - pb - pc);
                // order 0: G = |P_k0|, so P'_k0 = G' sign(P_k0)
                const float sg = (pa > 0.0f ? 1.0f : 0.0f) - (pa < 0.0f ? 1.0f : 0.0f);
                const float pa1 = ga * fmaf(sel0, sg, sel1 * 2.0f * pa);
                Ap[k][0] = pa1 + pd;
                Ap[k][1] = fmaf(c2b * gbc, pb, -pd);
                Ap[k][2] = fmaf(c2c * gbc, pc, -pd);
                Ap[k][3] = c2f * gf * pf;
            }
            // On a uniform grid B2 = k B1: for K <= 12 the factor k goes on the
            // atom's slices once (k P') instead of on every pair's B (12 fewer
            // multiplies per batch; at K = 16 the extra slices would spill)
            float Ak[KA ? K : 1][4];
            if constexpr (KA) {
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int q = 0; q < 4; ++q) Ak[k][q] = (float)k * Ap[k][q];
            }
            const int nb = aval ? a.cnt[(int64_t)b * a.n + p] : 0;
            int nbmax = nb;
            for (int off = 4; off < 64; off <<= 1) nbmax = max(nbmax, __shfl_xor(nbmax, off));
            // the same in every lane: the batch loop runs under the full EXEC
            // mask (the DPP broadcasts read every lane of a block)
            nbmax = __builtin_amdgcn_readfirstlane(nbmax);
            const int64_t row = (p * a.S + b) * a.cap;
            float w6[6] = {0, 0, 0, 0, 0, 0};
            // Software pipeline over batches of four pairs: while batch c0 runs,
            // the displacements of batch c0 + 4 are formed (LDS) and the list
            // entries of batch c0 + 12 are loaded.  Entry indices are clamped
            // into the row's slots; lanes past the row's length read the centre
            // atom (slot ip) and are inactive: unit displacement, zero B.
            const int cl = a.cap - 1;
            auto entry = [&](int c, int& q, int& im) {
                const int cc = min(c, cl);
                q = a.nbr[row + cc];
                im = a.img[row + cc];
            };
            auto geom = [&](int c, int q, int im, float& gdx, float& gdy, float& gdz, int& gslot, bool& gact) {
                const bool valid = c < nb;
                const int qq = valid ? q : (int)p;
                const int ii = valid ? im : kCentreWord;
                const float4 xj = pos.fetch(qq, ii, gslot);
                const float3 dm = pos.disp(xj, ii);
                gact = valid && dm.x * dm.x + dm.y * dm.y + dm.z * dm.z < a.rc2;  // skin entries carry no force
                gdx = gact ? dm.x : 1.0f;
                gdy = gact ? dm.y : 0.0f;
                gdz = gact ? dm.z : 0.0f;
            };
            float dx, dy, dz;
            int slot;
            bool act;
            int qA, iA, qB, iB;
            entry(j, qA, iA);
            geom(j, qA, iA, dx, dy, dz, slot, act);
            entry(4 + j, qA, iA);
            entry(8 + j, qB, iB);
            // one batch; (qx, ix) hold the entries of batch c0 + 4 and are
            // reloaded with those of batch c0 + 12
            auto batch = [&](int c0, int& qx, int& ix) {
                float ndx, ndy, ndz;
                int nslot;
                bool nact;
                geom(c0 + 4 + j, qx, ix, ndx, ndy, ndz, nslot, nact);
                entry(c0 + 12 + j, qx, ix);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float R = r2 * rinv;
                const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                float fc = 0.0f, dfc = 0.0f;
                if constexpr (RAD != kRadTab) {
                    const float ang = R * a.half_inv_rc;
                    fc = act ? 0.5f * __builtin_amdgcn_cosf(ang) + 0.5f : 0.0f;
                    dfc = act ? -0.5f * a.pi_over_rc * __builtin_amdgcn_sinf(ang) : 0.0f;
                }
                float B1[K], B2[K];
                if constexpr (RAD == kRadRec) {
                    const float t0 = R - mu0;
                    float ek = act ? __builtin_amdgcn_exp2f(nef0 * t0 * t0) : 0.0f;
                    float rk = __builtin_amdgcn_exp2f(fmaf(a.rec_a, t0, a.rec_b));
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        B1[k] = ek;
                        if constexpr (!KA) B2[k] = (float)k * ek;
                        ek *= rk;
                        rk *= a.rec_c;
                    }
                } else if constexpr (RAD == kRadTab) {
                    tabulated<K, true>(a, R, 0, B1, B2);
                    const float msk = act ? 1.0f : 0.0f;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        B1[k] *= msk;
                        B2[k] *= msk;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const float tk = R - a.mu[k];
                        const float e = __builtin_amdgcn_exp2f(-a.eta[k] * kLog2e * tk * tk);
                        B1[k] = e * fc;
                        B2[k] = e * fmaf(-2.0f * a.eta[k] * tk, fc, dfc);
                    }
                }
                f32x4 acc1[4], acc2[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc1[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                    acc2[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        acc1[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(Ap[k][q], B1[k], acc1[q], 0, 0, 0);
                        if constexpr (KA)
                            acc2[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(Ak[k][q], B1[k], acc2[q], 0, 0, 0);
                        else
                            acc2[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(Ap[k][q], B2[k], acc2[q], 0, 0, 0);
                    }
                }
                float V1[DR], V2[DR];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        V1[kMfmaRow[q][i]] = acc1[q][i];
                        V2[kMfmaRow[q][i]] = acc2[q][i];
                    }
                float Mv[DR];
                reduced_monomials<3>(ux, uy, uz, Mv);
                float S0 = 0.0f, S1 = 0.0f;
#pragma unroll
                for (int d = 0; d < DR; ++d) {
                    S0 = fmaf(Mv[d], V1[d], S0);
                    S1 = fmaf(Mv[d], V2[d], S1);
                }
                float Ax, Ay, Az, Bu;
                reduced_moment_adjoint<3>(ux, uy, uz, V1, Mv, Ax, Ay, Az, Bu);
                float sr, rf;
                if constexpr (RAD == kRadRec) {
                    sr = fmaf(a.rec_m2eta * fc, fmaf(-a.rec_delta, S1, (R - mu0) * S0), dfc * S0);
                    rf = rinv * fc;
                } else {
                    sr = S1;
                    rf = rinv;
                }
                if (act) {
                    const float gx = sr * ux + rf * (Ax - ux * Bu);
                    const float gy = sr * uy + rf * (Ay - uy * Bu);
                    const float gz = sr * uz + rf * (Az - uz * Bu);
                    Fo[0] += gx;
                    Fo[1] += gy;
                    Fo[2] += gz;
                    sink(slot, gx, gy, gz);
                    virial_add(w6, dx, dy, dz, gx, gy, gz);
                }
                dx = ndx;
                dy = ndy;
                dz = ndz;
                slot = nslot;
                act = nact;
            };
            int c0 = 0;
            for (; c0 + 8 <= nbmax; c0 += 8) {
                batch(c0, qA, iA);
                batch(c0 + 4, qB, iB);
            }
            if (c0 < nbmax) batch(c0, qA, iA);
            if (c0 + 4 < nbmax) batch(c0 + 4, qB, iB);
#pragma unroll
            for (int i = 0; i < 6; ++i) Wd[i] += (double)w6[i];
        }
        // the atom's own force: its four lanes' sums, added in a fixed order
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Fo[i] += __shfl_xor(Fo[i], 1);
            Fo[i] += __shfl_xor(Fo[i], 2);
        }
        if (aval && j == 0) {
            atomicAdd(&sF[ip], to_fixed(Fo[0]));
            atomicAdd(&sF[bg.hmax + ip], to_fixed(Fo[1]));
            atomicAdd(&sF[2 * bg.hmax + ip], to_fixed(Fo[2]));
        }
    }
    __syncthreads();
    for (int hc = wv; hc < nh; hc += kBlock / 64) {
        const int lo = h_base[hc], cnt = h_base[hc + 1] - lo;
        for (int k = lane; k < cnt; k += 64) {
            const int64_t q = h_first[hc] + k;
            const unsigned long long fx = sF[lo + k], fy = sF[bg.hmax + lo + k], fz = sF[2 * bg.hmax + lo + k];
            if (fx) atomicAdd(&bg.F[3 * q + 0], fx);
            if (fy) atomicAdd(&bg.F[3 * q + 1], fy);
            if (fz) atomicAdd(&bg.F[3 * q + 2], fz);
        }
    }
    block_virial(Wd, red, a.vir + (int64_t)blockIdx.x * kVirDoubles);
}

// Value of lane P of each block of four lanes, by a DPP quad permutation
// [P, P, P, P].
template <int P>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), P * 0x55, 0xF, 0xF, true));
}

// Descriptor on the matrix cores (M = 3, K = 4 KQ, blocked work order).  For
// an atom and a neighbour species, P = sum_c h(R_c) m(u_c)^T is a sum of one
// outer product per pair, taken as 4 x 4 x 1 FP32 MFMAs, one per (group kk of
// four radial functions, slice q of four kept components).  The four lanes of
// an MFMA block serve one atom (sixteen atoms per wave): lane j supplies the
// monomials of kept components kMfmaRow[q][j] as the A operand and h_{4 kk + j}
// as the B operand, so register i of its accumulator (kk, q) is
// P[4 kk + j][kMfmaRow[q][i]]: each lane ends with all sixteen kept
// components of its own radial functions and forms their G entries without
// any exchange.  The slices factor per lane as s, xx s, yy s and v s with
// s = (1, x, y, z)[j] and v = (xy, z, z, xy)[j].  Per batch each lane forms the
// geometry of one pair of its atom's row (entries and positions prefetched as
// in the matrix-core adjoint); the block's four pairs are then taken in turn,
// their unit vector, distance and cutoff weight broadcast by DPP.
template <int KQ, int RAD>
__global__ void __launch_bounds__(256, 2) k_descriptor_mfma(PathArgs a, BlockGeom bg) {
    constexpr int K = 4 * KQ, DR = Moments<3>::DR, D = Moments<3>::D;
    extern __shared__ __attribute__((aligned(8))) unsigned char lds_dyn[];
    __shared__ int32_t h_base[257], h_first[kMaxHaloCells], hoff[kMaxHaloCells];
    __shared__ int32_t wtmp[kBlock / 64];
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int quad = lane >> 2, j = lane & 3;
    const int blk = blockIdx.x;
    int x0, y0, z0;
    halo_slots(bg, blk, h_first, h_base, hoff, wtmp, x0, y0, z0);
    const int HX = bg.B[0] + 2, HY = bg.B[1] + 2;
    float* sx = reinterpret_cast<float*>(lds_dyn);
    float* sy = sx + bg.hmax;
    float* sz = sx + 2 * bg.hmax;
    halo_positions(bg, a, x0, y0, z0, h_first, h_base, sx, sy, sz);  // ends with a barrier
    const float cw[3] = {(float)(a.L[0] / bg.nc[0]), (float)(a.L[1] / bg.nc[1]), (float)(a.L[2] / bg.nc[2])};
    // this lane's monomial factors s = (1, x, y, z)[j] and v = (xy, z, z, xy)[j],
    // as 0/1 weights
    const float f1 = j == 0 ? 1.0f : 0.0f, fx = j == 1 ? 1.0f : 0.0f, fy = j == 2 ? 1.0f : 0.0f,
                fz = j == 3 ? 1.0f : 0.0f;
    const float vz = (j == 1 || j == 2) ? 1.0f : 0.0f, vxy = 1.0f - vz;
    // this lane's radial functions 4 kk + j
    float mu[KQ], nef[KQ];
#pragma unroll
    for (int kk = 0; kk < KQ; ++kk) {
        mu[kk] = a.mu[4 * kk + j];
        nef[kk] = -a.eta[4 * kk + j] * kLog2e;
    }
    const float ra4 = 4.0f * a.rec_a, rb4 = 16.0f * a.rec_b, rc4 = a.rec_c4;
    const int KM = K * 4;  // G features of one species
    const int64_t w0 = bg.wbase[blk];
    const int natoms = (int)(bg.wbase[blk + 1] - w0);
    for (int base = wv * 16; base < natoms; base += kBlock / 4) {
        const int ia = base + quad;
        const bool aval = ia < natoms;
        const int64_t w = w0 + (aval ? ia : natoms - 1);
        const int64_t g = bg.gbase[blk] + base / 16;
        const int64_t p = bg.wperm[w];
        const int ic = bg.wcell[w];
        const int ix = ic % bg.B[0] + 1, iy = (ic / bg.B[0]) % bg.B[1] + 1, iz = ic / (bg.B[0] * bg.B[1]) + 1;
        const int hp = (iz * HY + iy) * HX + ix;
        const int ip = hoff[hp] + (int)p;
        const LdsPos pos{sx, sy, sz, hoff, hp - (HX * HY + HX + 1), HX, HX * HY,
                         sx[ip] + cw[0], sy[ip] + cw[1], sz[ip] + cw[2], cw[0], cw[1], cw[2]};
        for (int b = 0; b < a.S; ++b) {
            f32x4 acc[KQ][4];
#pragma unroll
            for (int kk = 0; kk < KQ; ++kk)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[kk][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const int nb = aval ? a.cnt[(int64_t)b * a.n + p] : 0;
            int nbmax = nb;
            for (int off = 4; off < 64; off <<= 1) nbmax = max(nbmax, __shfl_xor(nbmax, off));
            // the same in every lane: the batch loop runs under the full EXEC
            // mask (the DPP broadcasts read every lane of a block)
            nbmax = __builtin_amdgcn_readfirstlane(nbmax);
            const int64_t row = (p * a.S + b) * a.cap;
            const int cl = a.cap - 1;
            auto entry = [&](int c, int& q, int& im) {
                const int cc = min(c, cl);
                q = a.nbr[row + cc];
                im = a.img[row + cc];
            };
            // lanes past the row's end read the centre atom and are inactive
            auto geom = [&](int c, int q, int im, float& gdx, float& gdy, float& gdz, bool& gact) {
                const bool valid = c < nb;
                int unused;
                const float4 xj = pos.fetch(valid ? q : (int)p, valid ? im : kCentreWord, unused);
                const float3 dm = pos.disp(xj, valid ? im : kCentreWord);
                gact = valid && dm.x * dm.x + dm.y * dm.y + dm.z * dm.z < a.rc2;  // skin entries add nothing
                gdx = gact ? dm.x : 1.0f;
                gdy = gact ? dm.y : 0.0f;
                gdz = gact ? dm.z : 0.0f;
            };
            float dx, dy, dz;
            bool act;
            int qA, iA, qB, iB;
            entry(j, qA, iA);
            geom(j, qA, iA, dx, dy, dz, act);
            entry(4 + j, qA, iA);
            entry(8 + j, qB, iB);
            // The MFMAs of pair P of the block.  The pair's lane hands over its
            // distance, weight and the products the slices share (each
            // broadcast feeds one arithmetic instruction, which takes it as a
            // DPP operand).
            struct PairVals {
                float R, wt, ux, uy, uz, xx, yy, xy;
            };
            auto pair_step = [&](auto pc, const PairVals& v) {
                constexpr int P = decltype(pc)::value;
                const float pR = quad_bcast<P>(v.R);
                float hB[KQ];
                if constexpr (RAD == kRadTab) {
                    const float xr = pR * a.tab_inv;
                    const float jf = fminf(floorf(xr), (float)a.tab_n);
                    const float tt = xr - jf;
                    const float4* trow = a.tab + (int64_t)jf * K + j;
                    float4 c[KQ];
#pragma unroll
                    for (int kk = 0; kk < KQ; ++kk) c[kk] = trow[4 * kk];
#pragma unroll
                    for (int kk = 0; kk < KQ; ++kk)
                        hB[kk] = fmaf(tt, fmaf(tt, fmaf(tt, c[kk].w, c[kk].z), c[kk].y), c[kk].x);
                } else if constexpr (RAD == kRadRec) {
                    // uniform grid: h_{k+4} = h_k r, r = exp2(4 rec_a t_k + 16 rec_b),
                    // and r gains the factor rec_c^16 per step of four
                    const float t0 = pR - mu[0];
                    float e = __builtin_amdgcn_exp2f(nef[0] * t0 * t0);
                    float r = __builtin_amdgcn_exp2f(fmaf(ra4, t0, rb4));
#pragma unroll
                    for (int kk = 0; kk < KQ; ++kk) {
                        hB[kk] = e;
                        e *= r;
                        r *= rc4;
                    }
                } else {
#pragma unroll
                    for (int kk = 0; kk < KQ; ++kk) {
                        const float tk = pR - mu[kk];
                        hB[kk] = __builtin_amdgcn_exp2f(nef[kk] * tk * tk);
                    }
                }
                // s = w (1, x, y, z)[j], then xx s, yy s and (z or xy) s.  The
                // lane's choices are 0/1 weights multiplying the broadcasts: a
                // select of a broadcast value may be compiled into a DPP move
                // under a partial EXEC mask, which reads the masked-off source
                // lane as zero.
                const float c = (quad_bcast<P>(v.ux) * fx + quad_bcast<P>(v.uy) * fy) + (quad_bcast<P>(v.uz) * fz + f1);
                const float sw = quad_bcast<P>(v.wt) * c;
                const float t3 = quad_bcast<P>(v.xy) * vxy + quad_bcast<P>(v.uz) * vz;
                const float Am[4] = {sw, quad_bcast<P>(v.xx) * sw, quad_bcast<P>(v.yy) * sw, t3 * sw};
#pragma unroll
                for (int kk = 0; kk < KQ; ++kk)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[kk][q] = __builtin_amdgcn_mfma_f32_4x4x1f32(Am[q], hB[kk], acc[kk][q], 0, 0, 0);
            };
            // one batch; (qx, ix) hold the entries of batch c0 + 4 and are
            // reloaded with those of batch c0 + 12
            auto batch = [&](int c0, int& qx, int& ix) {
                float ndx, ndy, ndz;
                bool nact;
                geom(c0 + 4 + j, qx, ix, ndx, ndy, ndz, nact);
                entry(c0 + 12 + j, qx, ix);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float R = r2 * rinv;
                const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                float wt;
                if constexpr (RAD == kRadTab) wt = act ? 1.0f : 0.0f;  // the table has the cutoff folded in
                else wt = act ? 0.5f * __builtin_amdgcn_cosf(R * a.half_inv_rc) + 0.5f : 0.0f;
                const PairVals v{R, wt, ux, uy, uz, ux * ux, uy * uy, ux * uy};
                pair_step(std::integral_constant<int, 0>{}, v);
                pair_step(std::integral_constant<int, 1>{}, v);
                pair_step(std::integral_constant<int, 2>{}, v);
                pair_step(std::integral_constant<int, 3>{}, v);
                dx = ndx;
                dy = ndy;
                dz = ndz;
                act = nact;
            };
            int c0 = 0;
            for (; c0 + 8 <= nbmax; c0 += 8) {
                batch(c0, qA, iA);
                batch(c0 + 4, qB, iB);
            }
            if (c0 < nbmax) batch(c0, qA, iA);
            if (c0 + 4 < nbmax) batch(c0 + 4, qB, iB);
            // P in the group layout (zeros for lanes past the block's atoms)
            if (a.Pbuf) {
                float* dst = a.Pbuf + (((int64_t)g * a.S + b) * K + j) * 256 + quad * 4;
#pragma unroll
                for (int kk = 0; kk < KQ; ++kk)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        __builtin_nontemporal_store(acc[kk][q], reinterpret_cast<f32x4*>(dst + kk * 1024 + q * 64));
            }
            if (aval) {
#pragma unroll
                for (int kk = 0; kk < KQ; ++kk) {
                    const int k = 4 * kk + j;
                    float Pr[1][DR], P[1][D];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int i = 0; i < 4; ++i) Pr[0][kMfmaRow[q][i]] = acc[kk][q][i];
                    expand_P<3, 1>(Pr, P);
                    float gv[4];
#pragma unroll
                    for (int m = 1; m <= 3; ++m) {
                        float sm = 0.0f;
#pragma unroll
                        for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) sm += kMult[d] * P[0][d] * P[0][d];
                        gv[m] = sm;
                    }
                    gv[0] = fabsf(P[0][0]);  // sqrt(S) of the single order-0 component
                    const int64_t gi = p * a.F + b * KM + 4 * k;
                    if (a.Gb) {
                        const bf16x4v h = {(__bf16)gv[0], (__bf16)gv[1], (__bf16)gv[2], (__bf16)gv[3]};
                        *reinterpret_cast<uint2*>(a.Gb + gi) = __builtin_bit_cast(uint2, h);
                    } else {
                        *reinterpret_cast<float4*>(a.G + gi) = make_float4(gv[0], gv[1], gv[2], gv[3]);
                    }
                }
            }
        }
    }
}

// Adjoint on the matrix cores for larger K (M = 3, K = 4 KS >= 24), one
// atom per wave at a time, its pairs sixteen at a time.  With E the group's
// radial functions (K x 16 pairs), V1 = P'^T E and V2 = (k P')^T E (on a
// uniform grid; else P'^T H and P'^T H') are 16 x 16 products over K, taken as
// v_mfma_f32_16x16x4f32 steps of four radial functions.  The A operand (row i
// = kept component, column = radial function 4 s + g from lane group g =
// lane / 16) stays in registers for the atom's whole row: K / 4 values of P'
// and of k P' per lane, formed from the atom-major P and dE/dG.  The B
// operand is the radial function 4 s + g of the lane's pair (pair = lane %
// 16).  Lane l ends with rows 4 g .. 4 g + 3 of its pair's column; row 4 g + r
// is kept component kMfmaRow[r][g], so a lane group holds the fold set
// s_g (1, xx, yy, v_g) of the 4x4x1 kernels: each lane forms its share of
// S0 = M.V1, S1 = M.V2 and A = sum_d V1_d grad M_d from its four rows, two
// exchanges (lanes 16 and 32 apart) complete them, lane groups 0, 1, 2
// scatter the force components x, y, z and group 3 adds the virial.
template <int KS, int RAD>
__global__ void __launch_bounds__(256, 2) k_adjoint_mfma16(PathArgs a, BlockGeom bg) {
    constexpr int K = 4 * KS, DR = Moments<3>::DR;
    extern __shared__ __attribute__((aligned(8))) unsigned char lds_dyn[];
    __shared__ int32_t h_base[257], h_first[kMaxHaloCells], hoff[kMaxHaloCells];
    __shared__ int32_t wtmp[kBlock / 64];
    __shared__ double red[6][kBlock / 64][2];
    __shared__ float2 rad_mm[RAD == kRadDirect ? K : 1];  // (mu_k, -2 eta_k)
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int jp = lane & 15, gq = lane >> 4;
    const int blk = blockIdx.x;
    int x0, y0, z0;
    halo_slots(bg, blk, h_first, h_base, hoff, wtmp, x0, y0, z0);
    const int HX = bg.B[0] + 2, HY = bg.B[1] + 2, HZ = bg.B[2] + 2;
    const int nh = HX * HY * HZ;
    const int hpos = (3 * bg.hmax + 1) & ~1;
    float* sx = reinterpret_cast<float*>(lds_dyn);
    float* sy = sx + bg.hmax;
    float* sz = sx + 2 * bg.hmax;
    unsigned long long* sF = reinterpret_cast<unsigned long long*>(sx + hpos);
    const int htot = h_base[nh];
    for (int i = t; i < htot; i += kBlock) {
        sF[i] = 0ull;
        sF[bg.hmax + i] = 0ull;
        sF[2 * bg.hmax + i] = 0ull;
    }
    if constexpr (RAD == kRadDirect)
        for (int k = t; k < K; k += kBlock) rad_mm[k] = make_float2(a.mu[k], -2.0f * a.eta[k]);
    halo_positions(bg, a, x0, y0, z0, h_first, h_base, sx, sy, sz);  // ends with a barrier
    const float cw[3] = {(float)(a.L[0] / bg.nc[0]), (float)(a.L[1] / bg.nc[1]), (float)(a.L[2] / bg.nc[2])};
    // A side: this lane supplies row jp = 4 gi + ri, kept component kMfmaRow[ri][gi]
    const int gi = jp >> 2, ri = jp & 3;
    // 2 x multiplicities in fold set gi (as in k_adjoint_mfma) and 0/1 weights
    const float c2b = gi <= 1 ? 2.0f : 6.0f;
    const float c2c = (gi & 1) ? 6.0f : 2.0f;
    const float c2f = gi == 3 ? 12.0f : 4.0f;
    const float c2d = (gi == 0 || gi == 3) ? 2.0f : 6.0f;
    const float sel0 = gi == 0 ? 1.0f : 0.0f, sel1 = 1.0f - sel0, sel3 = gi == 3 ? 1.0f : 0.0f, sel3c = 1.0f - sel3;
    const float wr0 = ri == 0 ? 1.0f : 0.0f, wr1 = ri == 1 ? 1.0f : 0.0f, wr2 = ri == 2 ? 1.0f : 0.0f,
                wr3 = ri == 3 ? 1.0f : 0.0f;
    // C side: this lane's rows are fold set gq, monomials s (1, xx, yy, v)
    const float f1 = gq == 0 ? 1.0f : 0.0f, fx = gq == 1 ? 1.0f : 0.0f, fy = gq == 2 ? 1.0f : 0.0f,
                fz = gq == 3 ? 1.0f : 0.0f;
    const float vz = (gq == 1 || gq == 2) ? 1.0f : 0.0f, vxy = 1.0f - vz;
    float mu_g = 0.0f, nef_g = 0.0f, mu0 = 0.0f;
    if constexpr (RAD == kRadRec) {
        mu_g = a.mu[gq];
        nef_g = -a.eta[gq] * kLog2e;
        mu0 = a.mu[0];
    }
    const float ra4 = 4.0f * a.rec_a, rb4 = 16.0f * a.rec_b, rc4 = a.rec_c4;
    const int64_t w0 = bg.wbase[blk];
    const int natoms = (int)(bg.wbase[blk + 1] - w0);
    double Wd[6] = {0, 0, 0, 0, 0, 0};
    for (int ia = wv; ia < natoms; ia += kBlock / 64) {
        const int64_t w = w0 + ia;
        const int64_t p = bg.wperm[w];
        const int ic = bg.wcell[w];
        const int ix = ic % bg.B[0] + 1, iy = (ic / bg.B[0]) % bg.B[1] + 1, iz = ic / (bg.B[0] * bg.B[1]) + 1;
        const int hp = (iz * HY + iy) * HX + ix;
        const int ip = hoff[hp] + (int)p;
        const LdsPos pos{sx, sy, sz, hoff, hp - (HX * HY + HX + 1), HX, HX * HY,
                         sx[ip] + cw[0], sy[ip] + cw[1], sz[ip] + cw[2], cw[0], cw[1], cw[2]};
        float Fo = 0.0f;  // component gq (< 3) of the centre atom's force, this lane's pairs
        for (int b = 0; b < a.S; ++b) {
            // this lane's A operands: P' (folded onto the kept basis) and k P'
            float A1[KS], A2[KS];
            const float* Pa = a.Pbuf + ((int64_t)w * a.S + b) * (K * DR);
            const float4* g4 = reinterpret_cast<const float4*>(a.dG + p * a.F + (int64_t)b * K * 4);
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                const int k = 4 * st + gq;
                const float4 pv = *reinterpret_cast<const float4*>(Pa + k * DR + 4 * gi);  // fold set gi
                const float pa = pv.x, pb = pv.y, pc = pv.z, pf = pv.w;
                const float4 g = g4[k];
                const float ga = fmaf(sel0, g.x, sel1 * g.y), gbc = fmaf(sel0, g.z, sel1 * g.w),
                            gf = fmaf(sel3, g.w, sel3c * g.z);
                const float pd = c2d * gbc * (pa - pb - pc);
                const float sg = (pa > 0.0f ? 1.0f : 0.0f) - (pa < 0.0f ? 1.0f : 0.0f);
                const float pa1 = ga * fmaf(sel0, sg, sel1 * 2.0f * pa);
                const float v0 = pa1 + pd, v1 = fmaf(c2b * gbc, pb, -pd), v2 = fmaf(c2c * gbc, pc, -pd),
                            v3 = c2f * gf * pf;
                A1[st] = fmaf(wr0, v0, fmaf(wr1, v1, fmaf(wr2, v2, wr3 * v3)));
                A2[st] = (float)k * A1[st];
            }
            const int nb = __builtin_amdgcn_readfirstlane(a.cnt[(int64_t)b * a.n + p]);
            const int64_t row = (p * a.S + b) * a.cap;
            float w6[6] = {0, 0, 0, 0, 0, 0};
            // Pipeline over the groups of sixteen pairs: while group c0 runs,
            // the displacements of group c0 + 16 are formed (LDS) and the list
            // entries of group c0 + 32 are loaded.  Entry indices are clamped
            // into the row's slots; columns past the row's end read the centre
            // atom and are inactive (unit displacement, zero B).
            const int cl = a.cap - 1;
            auto entry = [&](int c, int& q, int& im) {
                const int cc = min(c, cl);
                q = a.nbr[row + cc];
                im = a.img[row + cc];
            };
            auto geom = [&](int c, int q, int im, float& gdx, float& gdy, float& gdz, int& gslot, bool& gact) {
                const bool valid = c < nb;
                const int ii = valid ? im : kCentreWord;
                const float4 xj = pos.fetch(valid ? q : (int)p, ii, gslot);
                const float3 dm = pos.disp(xj, ii);
                gact = valid && dm.x * dm.x + dm.y * dm.y + dm.z * dm.z < a.rc2;
                gdx = gact ? dm.x : 1.0f;
                gdy = gact ? dm.y : 0.0f;
                gdz = gact ? dm.z : 0.0f;
            };
            float dx, dy, dz;
            int slot, qe, ie;
            bool act;
            entry(jp, qe, ie);
            geom(jp, qe, ie, dx, dy, dz, slot, act);
            entry(16 + jp, qe, ie);
            for (int c0 = 0; c0 < nb; c0 += 16) {
                float ndx, ndy, ndz;
                int nslot;
                bool nact;
                geom(c0 + 16 + jp, qe, ie, ndx, ndy, ndz, nslot, nact);
                entry(c0 + 32 + jp, qe, ie);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float R = r2 * rinv;
                const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                float fc = 0.0f, dfc = 0.0f;
                if constexpr (RAD != kRadTab) {
                    const float ang = R * a.half_inv_rc;
                    fc = act ? 0.5f * __builtin_amdgcn_cosf(ang) + 0.5f : 0.0f;
                    dfc = act ? -0.5f * a.pi_over_rc * __builtin_amdgcn_sinf(ang) : 0.0f;
                }
                // two accumulation chains per product (even and odd steps)
                f32x4 acc1 = {0.0f, 0.0f, 0.0f, 0.0f}, acc2 = {0.0f, 0.0f, 0.0f, 0.0f};
                f32x4 acc1b = {0.0f, 0.0f, 0.0f, 0.0f}, acc2b = {0.0f, 0.0f, 0.0f, 0.0f};
                auto step = [&](int st, float A1s, float A2s, float B1s, float B2s) {
                    if (st & 1) {
                        acc1b = __builtin_amdgcn_mfma_f32_16x16x4f32(A1s, B1s, acc1b, 0, 0, 0);
                        acc2b = __builtin_amdgcn_mfma_f32_16x16x4f32(A2s, B2s, acc2b, 0, 0, 0);
                    } else {
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(A1s, B1s, acc1, 0, 0, 0);
                        acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(A2s, B2s, acc2, 0, 0, 0);
                    }
                };
                if constexpr (RAD == kRadRec) {
                    // e_{4 s + g} by the stride-four recurrence, cutoff applied after
                    const float t0 = R - mu_g;
                    float e = act ? __builtin_amdgcn_exp2f(nef_g * t0 * t0) : 0.0f;
                    float rr = __builtin_amdgcn_exp2f(fmaf(ra4, t0, rb4));
#pragma unroll
                    for (int st = 0; st < KS; ++st) {
                        step(st, A1[st], A2[st], e, e);
                        e *= rr;
                        rr *= rc4;
                    }
                } else if constexpr (RAD == kRadTab) {
                    const float xr = R * a.tab_inv;
                    const float jf = fminf(floorf(xr), (float)a.tab_n);
                    const float tt = xr - jf;
                    const float4* trow = a.tab + (int64_t)jf * K + gq;
                    const float msk = act ? 1.0f : 0.0f;
#pragma unroll
                    for (int st = 0; st < KS; ++st) {
                        const float4 cf = trow[4 * st];
                        const float h = msk * fmaf(tt, fmaf(tt, fmaf(tt, cf.w, cf.z), cf.y), cf.x);
                        const float dh = msk * a.tab_inv * fmaf(tt, fmaf(3.0f * tt, cf.w, 2.0f * cf.z), cf.y);
                        step(st, A1[st], A1[st], h, dh);
                    }
                } else {
#pragma unroll
                    for (int st = 0; st < KS; ++st) {
                        const float2 mm = rad_mm[4 * st + gq];
                        const float tk = R - mm.x;
                        const float e = __builtin_amdgcn_exp2f(0.5f * kLog2e * mm.y * tk * tk);
                        step(st, A1[st], A1[st], e * fc, e * fmaf(mm.y * tk, fc, dfc));
                    }
                }
                acc1 += acc1b;
                acc2 += acc2b;
                // this lane's rows: V1, V2 at s (1, xx, yy, v) of fold set gq
                const float sm = fmaf(fx, ux, fmaf(fy, uy, fmaf(fz, uz, f1)));
                const float xx = ux * ux, yy = uy * uy, xy = ux * uy;
                const float vv = fmaf(vxy, xy, vz * uz);
                const float Q1 = fmaf(vv, acc1[3], fmaf(yy, acc1[2], fmaf(xx, acc1[1], acc1[0])));
                const float Q2 = fmaf(vv, acc2[3], fmaf(yy, acc2[2], fmaf(xx, acc2[1], acc2[0])));
                float S0 = sm * Q1, S1 = sm * Q2;
                float Ax = fmaf(fx, Q1, sm * fmaf(2.0f * ux, acc1[1], vxy * uy * acc1[3]));
                float Ay = fmaf(fy, Q1, sm * fmaf(2.0f * uy, acc1[2], vxy * ux * acc1[3]));
                float Az = fmaf(fz, Q1, sm * vz * acc1[3]);
#pragma unroll
                for (int off = 16; off <= 32; off <<= 1) {
                    S0 += __shfl_xor(S0, off);
                    S1 += __shfl_xor(S1, off);
                    Ax += __shfl_xor(Ax, off);
                    Ay += __shfl_xor(Ay, off);
                    Az += __shfl_xor(Az, off);
                }
                const float Bu = ux * Ax + uy * Ay + uz * Az;
                float sr, rf;
                if constexpr (RAD == kRadRec) {
                    sr = fmaf(a.rec_m2eta * fc, fmaf(-a.rec_delta, S1, (R - mu0) * S0), dfc * S0);
                    rf = rinv * fc;
                } else {
                    sr = S1;
                    rf = rinv;
                }
                const float gx = sr * ux + rf * (Ax - ux * Bu);
                const float gy = sr * uy + rf * (Ay - uy * Bu);
                const float gz = sr * uz + rf * (Az - uz * Bu);
                if (act) {
                    if (gq < 3) {
                        const float gc = gq == 0 ? gx : (gq == 1 ? gy : gz);
                        atomicAdd(&sF[gq * bg.hmax + slot], to_fixed(-gc));
                        Fo += gc;
                    } else {
                        virial_add(w6, dx, dy, dz, gx, gy, gz);
                    }
                }
                dx = ndx;
                dy = ndy;
                dz = ndz;
                slot = nslot;
                act = nact;
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) Wd[i] += (double)w6[i];
        }
        // the centre atom's force: each lane group's sixteen pair columns, fixed order
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) Fo += __shfl_xor(Fo, off);
        if (jp == 0 && gq < 3) atomicAdd(&sF[gq * bg.hmax + ip], to_fixed(Fo));
    }
    __syncthreads();
    for (int hc = wv; hc < nh; hc += kBlock / 64) {
        const int lo = h_base[hc], cnt = h_base[hc + 1] - lo;
        for (int k = lane; k < cnt; k += 64) {
            const int64_t q = h_first[hc] + k;
            const unsigned long long fx_ = sF[lo + k], fy_ = sF[bg.hmax + lo + k], fz_ = sF[2 * bg.hmax + lo + k];
            if (fx_) atomicAdd(&bg.F[3 * q + 0], fx_);
            if (fy_) atomicAdd(&bg.F[3 * q + 1], fy_);
            if (fz_) atomicAdd(&bg.F[3 * q + 2], fz_);
        }
    }
    block_virial(Wd, red, a.vir + (int64_t)blockIdx.x * kVirDoubles);
}

// ---- work order ----------------------------------------------------------
//
// Rows of one wave run in lockstep, so a wave costs the longest of its rows.
// In a two-species alloy the per-species row lengths of neighbouring atoms
// vary by several entries (the total hardly does), so each cell block's atoms
// are put in descending order of species-0 row length; the descriptor and
// adjoint kernels walk atoms in this order (and P is stored in it, which
// keeps its loads and stores coalesced).

struct WorkGeom {
    int nc[3], B[3], nb[3];
    const int32_t* cellstart;
    const int32_t* cnt;  // species-0 row lengths [n]
};

__device__ __forceinline__ void block_origin(const WorkGeom& g, int64_t blk, int& x0, int& y0, int& z0) {
    const int bx = (int)(blk % g.nb[0]), by = (int)((blk / g.nb[0]) % g.nb[1]), bz = (int)(blk / (g.nb[0] * g.nb[1]));
    x0 = bx * g.B[0];
    y0 = by * g.B[1];
    z0 = bz * g.B[2];
}

// Global cell index of interior cell ic of the block at (x0, y0, z0), or -1
// past the grid edge (the last block along an axis may be partial).
__device__ __forceinline__ int block_cell(const WorkGeom& g, int x0, int y0, int z0, int ic) {
    const int cx = x0 + ic % g.B[0], cy = y0 + (ic / g.B[0]) % g.B[1], cz = z0 + ic / (g.B[0] * g.B[1]);
    if (cx >= g.nc[0] || cy >= g.nc[1] || cz >= g.nc[2]) return -1;
    return (cz * g.nc[1] + cy) * g.nc[0] + cx;
}

// Atoms per block: one wave per block, lanes over its cells.
__global__ void k_wo_count(WorkGeom g, int64_t nblocks, int32_t* __restrict__ count) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (blk >= nblocks) return;  // whole wave
    int x0, y0, z0;
    block_origin(g, blk, x0, y0, z0);
    int c = 0;
    for (int ic = lane; ic < g.B[0] * g.B[1] * g.B[2]; ic += 64) {
        const int gc = block_cell(g, x0, y0, z0, ic);
        if (gc >= 0) c += g.cellstart[gc + 1] - g.cellstart[gc];
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane == 0) count[blk] = c;
}

// Exclusive scan of the block counts by one workgroup of 1024 threads;
// base[nblocks] = n.
__global__ void __launch_bounds__(1024) k_wo_scan(int64_t nblocks, const int32_t* __restrict__ count,
                                                  int32_t* __restrict__ base) {
    // base[0 .. nblocks] = exclusive scan of the counts (first work slots),
    // base[nblocks + 1 ..] = exclusive scan of ceil(count / 16) (first groups)
    __shared__ int32_t wsum[2][16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int32_t carry[2] = {0, 0};
    int32_t* gb = base + nblocks + 1;
    for (int64_t b0 = 0; b0 < nblocks; b0 += 1024) {
        const int64_t q = b0 + t;
        const int32_t c = q < nblocks ? count[q] : 0;
        const int32_t v[2] = {c, (c + 15) >> 4};
        int32_t x[2] = {v[0], v[1]};
        for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int32_t y = __shfl_up(x[u], off);
                if (lane >= off) x[u] += y;
            }
        }
        if (lane == 63) {
            wsum[0][wv] = x[0];
            wsum[1][wv] = x[1];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int32_t pre = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                const int32_t sw = wsum[u][w];
                pre += (w < wv) ? sw : 0;
                tot += sw;
            }
            if (q < nblocks) (u ? gb : base)[q] = carry[u] + pre + x[u] - v[u];
            carry[u] += tot;
        }
        __syncthreads();
    }
    if (t == 0) {
        base[nblocks] = carry[0];
        gb[nblocks] = carry[1];
    }
}

// One workgroup per block: counting sort of the block's atoms by descending
// species-0 row length (for one species, the row length).  In a two-species
// alloy the total row length hardly varies, so this orders the species-1 rows
// too.  Atoms of equal length land in arbitrary order.
__global__ void __launch_bounds__(256) k_wo_order(WorkGeom g, int cap, const int32_t* __restrict__ base,
                                                  int32_t* __restrict__ wperm, uint8_t* __restrict__ wcell) {
    extern __shared__ int32_t hist[];  // [cap + 2]: counts, then first slot per length; per-wave counts
    __shared__ int32_t i_base[257], i_first[kMaxBlockCells], wtmp[kBlock / 64];
    const int t = threadIdx.x;
    const int64_t blk = blockIdx.x;
    int x0, y0, z0;
    block_origin(g, blk, x0, y0, z0);
    const int nI = g.B[0] * g.B[1] * g.B[2];
    int icount = 0;
    if (t < nI) {
        const int gc = block_cell(g, x0, y0, z0, t);
        i_first[t] = gc >= 0 ? g.cellstart[gc] : 0;
        icount = gc >= 0 ? g.cellstart[gc + 1] - i_first[t] : 0;
    }
    for (int k = t; k < (cap + 2) + (kBlock / 64) * (cap + 1); k += kBlock) hist[k] = 0;
    scan256(icount, i_base, wtmp);  // ends with a barrier
    const int m = i_base[nI];
    for (int la = t; la < m; la += kBlock) {
        int ic = 0;
        while (ic + 1 < nI && i_base[ic + 1] <= la) ++ic;
        const int len = min(g.cnt[i_first[ic] + (la - i_base[ic])], cap);
        atomicAdd(&hist[len], 1);
    }
    __syncthreads();
    if (t == 0) {  // descending lengths: first slot of length L = atoms longer than L
        int run = 0;
        for (int L = cap; L >= 0; --L) {
            const int c = hist[L];
            hist[L] = run;
            run += c;
        }
    }
    __syncthreads();
    // Slots in a fixed order: atoms of equal length keep their cell order.
    // Rounds of kBlock atoms; an atom's slot is its length's running first
    // slot plus the number of earlier atoms of the round with that length:
    // the lanes before it in its wave (ballots) and the earlier waves' counts
    // of that length (LDS histograms per wave, whose totals do not depend on
    // the order of the atomics).
    const int lane = t & 63, wvi = t >> 6;
    int32_t* whist = hist + cap + 2;  // [kBlock / 64][cap + 1]
    const int64_t w0 = base[blk];
    for (int r0 = 0; r0 < m; r0 += kBlock) {
        const int la = r0 + t;
        int ic = 0, len = -1;
        int64_t p = 0;
        if (la < m) {
            while (ic + 1 < nI && i_base[ic + 1] <= la) ++ic;
            p = i_first[ic] + (la - i_base[ic]);
            len = min(g.cnt[p], cap);
        }
        int before = 0;
        unsigned long long todo = __ballot(len >= 0);
        while (todo) {  // the same in every lane: one pass per distinct length
            const int lv = __shfl(len, __builtin_ctzll(todo));
            const unsigned long long grp = __ballot(len == lv);
            if (len == lv) before = __popcll(grp & ((1ull << lane) - 1));
            todo &= ~grp;
        }
        if (len >= 0) atomicAdd(&whist[wvi * (cap + 1) + len], 1);
        __syncthreads();
        if (len >= 0) {
            for (int u = 0; u < wvi; ++u) before += whist[u * (cap + 1) + len];
            const int slot = hist[len] + before;
            wperm[w0 + slot] = (int32_t)p;
            wcell[w0 + slot] = (uint8_t)ic;
        }
        __syncthreads();  // every lane has its slot
        for (int L = t; L <= cap; L += kBlock) {
            int c = 0;
            for (int u = 0; u < kBlock / 64; ++u) {
                c += whist[u * (cap + 1) + L];
                whist[u * (cap + 1) + L] = 0;
            }
            hist[L] += c;
        }
        __syncthreads();  // hist and whist are reused by the next round
    }
}

__global__ void k_zero(unsigned long long* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

using PathFn = void (*)(PathArgs, int64_t);
using AtomicFn = void (*)(PathArgs, unsigned long long*);
using BlockedFn = void (*)(PathArgs, BlockGeom);

template <int KC, bool TAB, int PL>
PathFn pick_desc_nt(int M) {
    switch (M) {
        case 0: return k_descriptor<KC, 0, TAB, PL>;
        case 1: return k_descriptor<KC, 1, TAB, PL>;
        case 2: return k_descriptor<KC, 2, TAB, PL>;
        default: return k_descriptor<KC, 3, TAB, PL>;
    }
}
// pl 2 (atom-major P) only for M = 3 with chunks of four or six
template <int KC, bool TAB>
PathFn pick_desc(int M, int pl) {
    if constexpr (KC == 4 || KC == 6)
        if (pl == 2) return k_descriptor<KC, 3, TAB, 2>;
    return pl == 1 ? pick_desc_nt<KC, TAB, 1>(M) : pick_desc_nt<KC, TAB, 0>(M);
}
template <int KC, int RAD>
AtomicFn pick_atomic(int M) {
    switch (M) {
        case 0: return k_adjoint_atomic<KC, 0, RAD>;
        case 1: return k_adjoint_atomic<KC, 1, RAD>;
        case 2: return k_adjoint_atomic<KC, 2, RAD>;
        default: return k_adjoint_atomic<KC, 3, RAD>;
    }
}
template <int KC, int RAD, bool PAIR2>
BlockedFn pick_blocked_p(int M) {
    switch (M) {
        case 0: return k_adjoint_blocked<KC, 0, RAD, PAIR2>;
        case 1: return k_adjoint_blocked<KC, 1, RAD, PAIR2>;
        case 2: return k_adjoint_blocked<KC, 2, RAD, PAIR2>;
        default: return k_adjoint_blocked<KC, 3, RAD, PAIR2>;
    }
}
// Two chunk lanes per atom happen only with chunks of 6 or 8 (K = 12, 16).
template <int KC, int RAD>
BlockedFn pick_blocked(int M, bool pair2) {
    if constexpr (KC >= 6)
        if (pair2) return pick_blocked_p<KC, RAD, true>(M);
    return pick_blocked_p<KC, RAD, false>(M);
}

template <bool TAB>
PathFn select_desc(int kc, int M, int pl) {
    switch (kc) {
        case 3: return pick_desc<3, TAB>(M, pl);
        case 4: return pick_desc<4, TAB>(M, pl);
        case 6: return pick_desc<6, TAB>(M, pl);
        default: return pick_desc<8, TAB>(M, pl);
    }
}
template <int RAD>
AtomicFn select_atomic_r(int kc, int M) {
    switch (kc) {
        case 4: return pick_atomic<4, RAD>(M);
        case 6: return pick_atomic<6, RAD>(M);
        default: return pick_atomic<8, RAD>(M);
    }
}
AtomicFn select_atomic(int rad, int kc, int M) {
    return rad == kRadTab ? select_atomic_r<kRadTab>(kc, M)
                          : rad == kRadRec ? select_atomic_r<kRadRec>(kc, M) : select_atomic_r<kRadDirect>(kc, M);
}
template <int RAD>
BlockedFn select_blocked_r(int kc, int M, bool pair2) {
    switch (kc) {
        case 4: return pick_blocked<4, RAD>(M, pair2);
        case 6: return pick_blocked<6, RAD>(M, pair2);
        default: return pick_blocked<8, RAD>(M, pair2);
    }
}
template <int RAD>
BlockedFn select_mfma_r(int kq) {
    switch (kq) {
        case 2: return k_adjoint_mfma<2, RAD>;
        case 3: return k_adjoint_mfma<3, RAD>;
        default: return k_adjoint_mfma<4, RAD>;
    }
}
BlockedFn select_mfma(int rad, int kq) {
    return rad == kRadTab ? select_mfma_r<kRadTab>(kq)
                          : rad == kRadRec ? select_mfma_r<kRadRec>(kq) : select_mfma_r<kRadDirect>(kq);
}
// The matrix-core adjoint takes M = 3 and K = 8, 12 or 16 (K / 4 slices of
// P' per lane stay in registers); so does the matrix-core descriptor.
bool mfma_adjoint(const tmd_model* m) { return m->M == 3 && m->K % 4 == 0 && m->K >= 8 && m->K <= 16; }

template <int RAD>
BlockedFn select_desc_mfma_r(int kq) {
    switch (kq) {
        case 2: return k_descriptor_mfma<2, RAD>;
        case 3: return k_descriptor_mfma<3, RAD>;
        default: return k_descriptor_mfma<4, RAD>;
    }
}
template <int RAD>
BlockedFn select_mfma16_r(int ks) {
    switch (ks) {
        case 6: return k_adjoint_mfma16<6, RAD>;
        case 8: return k_adjoint_mfma16<8, RAD>;
        case 12: return k_adjoint_mfma16<12, RAD>;
        case 16: return k_adjoint_mfma16<16, RAD>;
        case 24: return k_adjoint_mfma16<24, RAD>;
        default: return k_adjoint_mfma16<32, RAD>;
    }
}
BlockedFn select_mfma16(int rad, int ks) {
    return rad == kRadTab ? select_mfma16_r<kRadTab>(ks)
                          : rad == kRadRec ? select_mfma16_r<kRadRec>(ks) : select_mfma16_r<kRadDirect>(ks);
}

BlockedFn select_desc_mfma(int rad, int kq) {
    return rad == kRadTab ? select_desc_mfma_r<kRadTab>(kq)
                          : rad == kRadRec ? select_desc_mfma_r<kRadRec>(kq) : select_desc_mfma_r<kRadDirect>(kq);
}

BlockedFn select_blocked(int rad, int kc, int M, bool pair2) {
    return rad == kRadTab ? select_blocked_r<kRadTab>(kc, M, pair2)
                          : rad == kRadRec ? select_blocked_r<kRadRec>(kc, M, pair2)
                                           : select_blocked_r<kRadDirect>(kc, M, pair2);
}

PathArgs make_args(const tmd_model* m, const tmd_nlist* nl) {
    PathArgs a{};
    a.n = nl->n;
    a.S = m->S;
    a.K = m->K;
    a.F = m->F;
    a.cap = nl->cap;
    int nch = m->K / m->kc, lg = 0;
    while ((1 << lg) < nch) ++lg;
    a.nch_log2 = lg;
    const double rc = m->rcut;
    a.rc2 = (float)(rc * rc);
    a.half_inv_rc = (float)(0.5 / rc);
    a.pi_over_rc = (float)(M_PI / rc);
    a.rec = m->rec ? 1 : 0;
    a.rec_a = m->rec_a;
    a.rec_b = m->rec_b;
    a.rec_c = m->rec_c;
    a.rec_c4 = m->rec_c4;
    a.rec_m2eta = m->rec ? (float)(-2.0 * m->eta_h[0]) : 0.0f;
    a.rec_delta = m->rec ? (float)(m->mu_h[1] - m->mu_h[0]) : 0.0f;
    a.tab = m->tab;
    a.tab_inv = m->tab ? (float)(1.0 / m->tab_delta) : 0.0f;
    a.tab_n = m->tab_n;
    for (int q = 0; q < 3; ++q) a.L[q] = nl->box[q];
    a.boxes = nl->boxes;
    a.xs = nl->xs;
    a.nbr = nl->nbr;
    a.img = nl->img;
    a.cnt = nl->cnt;
    a.wperm = nl->wo_valid ? nl->wperm : nullptr;
    a.mu = m->mu;
    a.eta = m->eta;
    return a;
}

unsigned path_grid(const tmd_model* m, const tmd_nlist* nl) {
    const int64_t threads = nl->n * (m->K / m->kc);
    return (unsigned)((threads + kBlock - 1) / kBlock);
}

// Radial functions per descriptor thread.  P is stored per radial function,
// so the descriptor's chunking need not match the adjoint's (m->kc).
// Measured: four per thread beat eight for K = 32 and 128 with M = 3.
int desc_kc(const tmd_model* m) { return (m->M == 3 && m->kc == 8) ? 4 : m->kc; }

// The 16x16x4 matrix-core adjoint takes M = 3 and K = 24 .. 128 (K / 4 steps
// of four radial functions), reading P in the atom-major layout that the
// descriptor writes with chunks of four or six.
bool mfma16_adjoint(const tmd_model* m) {
    const int kcd = desc_kc(m);
    return m->M == 3 && m->K >= 24 && m->K <= 128 && m->K % 4 == 0 && (kcd == 4 || kcd == 6);
}

int log2_int(int v) {
    int lg = 0;
    while ((1 << lg) < v) ++lg;
    return lg;
}

// Per halo atom the blocked adjoint keeps its position (3 floats) and its
// fixed-point force accumulators (3 x 8 bytes) in LDS; capped so that two
// workgroups fit on a CU.
constexpr size_t kHaloBytes = 3 * sizeof(float) + 3 * sizeof(unsigned long long);
constexpr size_t kMaxDynLds = 76 * 1024;
size_t blocked_lds_bytes(int hmax) { return sizeof(float) * (size_t)((3 * hmax + 1) & ~1) + 24 * (size_t)hmax; }

// Block geometry of the work order of a built list.
BlockGeom wo_geom(const tmd_nlist* nl) {
    BlockGeom bg{};
    for (int d = 0; d < 3; ++d) {
        bg.nc[d] = nl->nc[d];
        bg.B[d] = nl->wo_B[d];
        bg.nb[d] = nl->wo_nb[d];
    }
    bg.hmax = nl->wo_hmax;
    bg.cellstart = nl->cellstart;
    bg.wbase = nl->wbase;
    bg.gbase = nl->wbase + ((int64_t)nl->wo_nb[0] * nl->wo_nb[1] * nl->wo_nb[2] + 1);
    bg.wperm = nl->wperm;
    bg.wcell = nl->wcell;
    return bg;
}

// Largest block shape whose halo accumulators fit in LDS for the densest cell.
bool choose_blocks(const tmd_nlist* nl, BlockGeom* bg) {
    // 4x4x2 cells per workgroup (about 2,500 workgroups at 1 M atoms, several
    // rounds per CU; its halo of 4.5 cells per interior cell fits the LDS
    // budget at r_c = 6 A), then 4x2x2 and 3x2x2 for denser or larger cells.
    // The largest halos of these three are counted exactly during the build;
    // the other fallbacks use (halo cells) x (densest cell).
    static const int shapes[][3] = {{kBlockShape[0], kBlockShape[1], kBlockShape[2]},
                                    {kBlockShape2[0], kBlockShape2[1], kBlockShape2[2]},
                                    {kBlockShape3[0], kBlockShape3[1], kBlockShape3[2]},
                                    {2, 2, 2},
                                    {2, 2, 1},
                                    {2, 1, 1},
                                    {1, 1, 1}};
    for (const auto& sh : shapes) {
        int B[3], H = 1;
        for (int d = 0; d < 3; ++d) {
            B[d] = std::min(sh[d], nl->nc[d]);
            H *= B[d] + 2;
        }
        const bool last = &sh == &shapes[6];
        const int counted = &sh == &shapes[0]   ? nl->halo_max
                            : &sh == &shapes[1] ? nl->halo_max2
                            : &sh == &shapes[2] ? nl->halo_max3
                                                : -1;
        const int64_t hmax = counted >= 0 ? (int64_t)std::max(1, counted) : (int64_t)H * std::max(1, nl->max_occ);
        // small systems: smaller blocks until every CU gets two workgroups
        int64_t nblocks = 1;
        for (int d = 0; d < 3; ++d) nblocks *= (nl->nc[d] + B[d] - 1) / B[d];
        if (!last && nblocks < 2 * (int64_t)nl->ctx->num_cus) continue;
        if ((int64_t)blocked_lds_bytes((int)std::min<int64_t>(hmax, 1 << 20)) > (int64_t)kMaxDynLds) continue;
        for (int d = 0; d < 3; ++d) {
            bg->nc[d] = nl->nc[d];
            bg->B[d] = B[d];
            bg->nb[d] = (nl->nc[d] + B[d] - 1) / B[d];
        }
        bg->hmax = (int)hmax;
        return true;
    }
    return false;
}

}  // namespace

constexpr size_t kWoOrderMaxLds = 48 * 1024;

tmd_status launch_work_order(tmd_context* ctx, tmd_nlist* nl) {
    nl->wo_valid = false;
    BlockGeom bg{};
    if (!nl->narrow || !choose_blocks(nl, &bg)) return TMD_OK;  // atomic adjoint, identity order
    const int64_t nblocks = (int64_t)bg.nb[0] * bg.nb[1] * bg.nb[2];
    if (nl->wbase_cap < 2 * (nblocks + 1)) {
        if (nl->wbase) TMD_HIP(ctx, hipFree(nl->wbase));
        nl->wbase = nullptr;
        nl->wbase_cap = 0;
        TMD_HIP(ctx, hipMalloc((void**)&nl->wbase, sizeof(int32_t) * 2 * (nblocks + 1)));
        nl->wbase_cap = 2 * (nblocks + 1);
    }
    hipError_t e = hipSuccess;
    int32_t* count = (int32_t*)ctx->ws.get("wo.count", sizeof(int32_t) * nblocks, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "work order workspace");
    WorkGeom g{};
    for (int d = 0; d < 3; ++d) {
        g.nc[d] = bg.nc[d];
        g.B[d] = bg.B[d];
        g.nb[d] = bg.nb[d];
    }
    g.cellstart = nl->cellstart;
    g.cnt = nl->cnt;
    // length histograms in LDS: one counter per possible row length, for the
    // block and for each of its waves (rows longer than ~2,400 entries would
    // need more than 48 KB: no work order, the atomic adjoint instead)
    const size_t lds = sizeof(int32_t) * (((size_t)nl->cap + 2) + (kBlock / 64) * ((size_t)nl->cap + 1));
    if (lds > kWoOrderMaxLds) return TMD_OK;
    {
        ProfScope ps_(ctx, "work_order");
        k_wo_count<<<(unsigned)((nblocks + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, ctx->stream>>>(g, nblocks,
                                                                                                   count);
        k_wo_scan<<<1, 1024, 0, ctx->stream>>>(nblocks, count, nl->wbase);
        k_wo_order<<<(unsigned)nblocks, kBlock, lds, ctx->stream>>>(g, nl->cap, nl->wbase, nl->wperm, nl->wcell);
    }
    TMD_HIP(ctx, hipGetLastError());
    for (int d = 0; d < 3; ++d) {
        nl->wo_B[d] = bg.B[d];
        nl->wo_nb[d] = bg.nb[d];
    }
    nl->wo_hmax = bg.hmax;
    nl->wo_valid = true;
    return TMD_OK;
}

int64_t p_slots(const tmd_model* m, const tmd_nlist* nl) {
    if (!(nl->wo_valid && mfma_adjoint(m))) return nl->n;
    // each block's last group may be partly empty
    const int64_t nblocks = (int64_t)nl->wo_nb[0] * nl->wo_nb[1] * nl->wo_nb[2];
    return nl->n + 15 * std::min<int64_t>(nblocks, nl->n);
}

int64_t p_slots_reserve(int64_t n) { return n + n / 8 + 16 * 1024; }

int64_t adjoint_max_partials(const tmd_model* m, const tmd_nlist* nl) {
    return std::max<int64_t>((int64_t)path_grid(m, nl), nl->ncells);
}

tmd_status launch_descriptors(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, float* G, float* Pbuf,
                              uint16_t* Gb) {
    PathArgs a = make_args(m, nl);
    a.G = G;
    a.Gb = Gb;
    a.Pbuf = Pbuf;
    if (nl->wo_valid && mfma_adjoint(m)) {
        const BlockGeom bg = wo_geom(nl);
        const unsigned grid = (unsigned)bg.nb[0] * bg.nb[1] * bg.nb[2];
        auto fn = select_desc_mfma(m->tab ? kRadTab : (m->rec4 ? kRadRec : kRadDirect), m->K / 4);
        const size_t lds = sizeof(float) * 3 * (size_t)bg.hmax;  // halo positions
        {
            ProfScope ps_(ctx, "descriptor");
            fn<<<grid, kBlock, lds, ctx->stream>>>(a, bg);
        }
        TMD_HIP(ctx, hipGetLastError());
        return TMD_OK;
    }
    const int kcd = desc_kc(m);
    a.nch_log2 = log2_int(m->K / kcd);
    // P stores cover whole 128-byte lines (and go out non-temporally) with at most two chunks per atom
    // atom-major P for the 16x16x4 adjoint; else element-major, non-temporal
    // when the stores cover whole lines
    const int pl = (nl->wo_valid && mfma16_adjoint(m)) ? 2 : (a.nch_log2 <= 1 ? 1 : 0);
    auto fn = m->tab ? select_desc<true>(kcd, m->M, pl) : select_desc<false>(kcd, m->M, pl);
    const int64_t nblocks = (nl->n * (m->K / kcd) + kBlock - 1) / kBlock;
    {
        ProfScope ps_(ctx, "descriptor");
        fn<<<xcd_grid(nblocks), kBlock, 0, ctx->stream>>>(a, nblocks);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_adjoint(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, const float* dG, float* Pbuf,
                          unsigned long long* Fsorted, double* vir_partials, int* nvir_out) {
    PathArgs a = make_args(m, nl);
    a.dG = dG;
    a.Pbuf = Pbuf;
    a.vir = vir_partials;
    // zeroed by a kernel rather than a memset, so that the sequence can be
    // captured into a graph and replayed
    k_zero<<<(unsigned)((3 * nl->n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(Fsorted, 3 * nl->n);
    if (nl->wo_valid) {
        BlockGeom bg = wo_geom(nl);
        bg.F = Fsorted;
        const unsigned grid = (unsigned)bg.nb[0] * bg.nb[1] * bg.nb[2];
        // P's layout does not depend on the chunk: for M = 3 and K >= 64 four
        // radial functions per lane (two waves per SIMD) beat eight (one wave;
        // measured at K = 128: 0.947 -> 0.908 ms; at K = 32 eight stay faster,
        // 0.600 against 0.636 ms)
        const int kca = (m->M == 3 && m->kc == 8 && m->K >= 64) ? 4 : m->kc;
        a.nch_log2 = log2_int(m->K / kca);
        const bool pair2 = m->K / kca == 2;  // two chunk lanes per atom share the pair geometry
        const int rad = m->tab ? kRadTab : (m->rec ? kRadRec : kRadDirect);
        const int rad4 = m->tab ? kRadTab : (m->rec4 ? kRadRec : kRadDirect);  // stride-four recurrence
        auto fn = mfma_adjoint(m)     ? select_mfma(rad, m->K / 4)
                  : mfma16_adjoint(m) ? select_mfma16(rad4, m->K / 4)
                                      : select_blocked(rad, kca, m->M, pair2);
        {
            ProfScope ps_(ctx, "adjoint");
            fn<<<grid, kBlock, blocked_lds_bytes(bg.hmax), ctx->stream>>>(a, bg);
        }
        *nvir_out = (int)grid;
    } else {
        const unsigned grid = path_grid(m, nl);
        const int rad = m->tab ? kRadTab : (m->rec ? kRadRec : kRadDirect);
        auto fn = select_atomic(rad, m->kc, m->M);
        {
            ProfScope ps_(ctx, "adjoint");
            fn<<<grid, kBlock, 0, ctx->stream>>>(a, Fsorted);
        }
        *nvir_out = (int)grid;
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd
