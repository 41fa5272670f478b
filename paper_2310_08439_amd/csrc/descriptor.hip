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
// neighbours from the column-major list, recomputing the pair geometry.  No
// intermediate per-pair tensor is stored: the only HBM traffic is the list,
// the positions (gathered, cache-resident), G / dG and the outputs.
// Per-pair force partials of the chunks are summed with lane shuffles.
#include "tmd_internal.h"

namespace tmd {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

template <int M>
struct Moments {
    static constexpr int D = (M + 1) * (M + 2) * (M + 3) / 6;
};

// Multiplicity of moment component d (T_dm row order: 1; x y z; xx xy xz yy
// yz zz; xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz).
__device__ constexpr float kMult[20] = {1, 1, 1, 1, 1, 2, 2, 1, 2, 1, 1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
__device__ constexpr int kOrderStart[5] = {0, 1, 4, 10, 20};

template <int M>
__device__ __forceinline__ void monomials(float x, float y, float z, float* Mv) {
    Mv[0] = 1.0f;
    if constexpr (M >= 1) {
        Mv[1] = x;
        Mv[2] = y;
        Mv[3] = z;
    }
    if constexpr (M >= 2) {
        Mv[4] = x * x;
        Mv[5] = x * y;
        Mv[6] = x * z;
        Mv[7] = y * y;
        Mv[8] = y * z;
        Mv[9] = z * z;
    }
    if constexpr (M >= 3) {
        Mv[10] = Mv[4] * x;
        Mv[11] = Mv[4] * y;
        Mv[12] = Mv[4] * z;
        Mv[13] = x * Mv[7];
        Mv[14] = x * Mv[8];
        Mv[15] = x * Mv[9];
        Mv[16] = Mv[7] * y;
        Mv[17] = Mv[7] * z;
        Mv[18] = y * Mv[9];
        Mv[19] = Mv[9] * z;
    }
}

// A = sum_d V_d grad_u M_d and B = sum_d ord(d) V_d M_d.
template <int M>
__device__ __forceinline__ void moment_adjoint(float x, float y, float z, const float* V, const float* Mv,
                                               float& Ax, float& Ay, float& Az, float& B) {
    Ax = Ay = Az = 0.0f;
    B = 0.0f;
    if constexpr (M >= 1) {
        Ax = V[1];
        Ay = V[2];
        Az = V[3];
        B = V[1] * x + V[2] * y + V[3] * z;
    }
    if constexpr (M >= 2) {
        Ax += 2.0f * x * V[4] + y * V[5] + z * V[6];
        Ay += x * V[5] + 2.0f * y * V[7] + z * V[8];
        Az += x * V[6] + y * V[8] + 2.0f * z * V[9];
        float b2 = 0.0f;
#pragma unroll
        for (int d = 4; d < 10; ++d) b2 += V[d] * Mv[d];
        B += 2.0f * b2;
    }
    if constexpr (M >= 3) {
        const float xx = Mv[4], xy = Mv[5], xz = Mv[6], yy = Mv[7], yz = Mv[8], zz = Mv[9];
        Ax += 3.0f * xx * V[10] + 2.0f * xy * V[11] + 2.0f * xz * V[12] + yy * V[13] + yz * V[14] + zz * V[15];
        Ay += xx * V[11] + 2.0f * xy * V[13] + xz * V[14] + 3.0f * yy * V[16] + 2.0f * yz * V[17] + zz * V[18];
        Az += xx * V[12] + xy * V[14] + 2.0f * xz * V[15] + yy * V[17] + 2.0f * yz * V[18] + 3.0f * zz * V[19];
        float b3 = 0.0f;
#pragma unroll
        for (int d = 10; d < 20; ++d) b3 += V[d] * Mv[d];
        B += 3.0f * b3;
    }
}

struct PathArgs {
    int64_t n;
    int S, K, F, cap, nch_log2;
    float rc2, half_inv_rc, pi_over_rc;
    double L[3];
    const double4* xs;
    const int32_t* nbr;
    const int32_t* img;
    const int32_t* cnt;
    const float* mu;
    const float* eta;
    // forward output / backward input
    float* G;
    const float* dG;
    // backward outputs
    float* Fown;
    float* Fin;
    double* vir;
};

struct Pair {
    float dx, dy, dz, r2;
    int q;  // neighbour (sorted index)
};

// NB consecutive list entries c0 .. c0+NB-1 of a row of nb (>= 1) entries:
// all index loads are issued before all position loads so that they overlap.
// Entries past the row end repeat the last valid entry (never a stale slot)
// and are marked with r2 = +inf so that every consumer skips them.
template <int NB>
__device__ __forceinline__ void load_pairs(const PathArgs& a, const double4& xi, int64_t base, int c0, int nb,
                                           Pair (&pr)[NB]) {
    int q[NB], im[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int64_t slot = base + (int64_t)min(c0 + j, nb - 1) * a.n;
        q[j] = a.nbr[slot];
        im[j] = a.img[slot];
    }
    double4 xj[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) xj[j] = a.xs[q[j]];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        int nx, ny, nz;
        unpack_img(im[j], nx, ny, nz);
        pr[j].dx = (float)((xj[j].x - xi.x) + (double)nx * a.L[0]);
        pr[j].dy = (float)((xj[j].y - xi.y) + (double)ny * a.L[1]);
        pr[j].dz = (float)((xj[j].z - xi.z) + (double)nz * a.L[2]);
        pr[j].r2 = (c0 + j < nb) ? pr[j].dx * pr[j].dx + pr[j].dy * pr[j].dy + pr[j].dz * pr[j].dz
                                 : __builtin_inff();
        pr[j].q = q[j];
    }
}

constexpr int kBatchFwd = 4;
constexpr int kBatchAdj = 2;

// P tile of one species for this thread's radial chunk.
template <int KC, int M>
__device__ __forceinline__ void accumulate_P(const PathArgs& a, const double4& xi, int64_t p, int b,
                                             const float* mu, const float* nef, float (&P)[KC][Moments<M>::D]) {
    constexpr int D = Moments<M>::D;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
        for (int d = 0; d < D; ++d) P[kk][d] = 0.0f;
    const int nb = a.cnt[(int64_t)b * a.n + p];
    const int64_t base = (int64_t)b * a.cap * a.n + p;
    for (int c0 = 0; c0 < nb; c0 += kBatchFwd) {
      Pair prs[kBatchFwd];
      load_pairs<kBatchFwd>(a, xi, base, c0, nb, prs);
#pragma unroll
      for (int j = 0; j < kBatchFwd; ++j) {
        const Pair& pr = prs[j];
        if (pr.r2 >= a.rc2) continue;
        const float rinv = __builtin_amdgcn_rsqf(pr.r2);
        const float R = pr.r2 * rinv;
        const float ux = pr.dx * rinv, uy = pr.dy * rinv, uz = pr.dz * rinv;
        const float fc = 0.5f * __builtin_amdgcn_cosf(R * a.half_inv_rc) + 0.5f;
        float Mv[D];
        monomials<M>(ux, uy, uz, Mv);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const float t = R - mu[kk];
            const float h = __builtin_amdgcn_exp2f(nef[kk] * t * t) * fc;
#pragma unroll
            for (int d = 0; d < D; ++d) P[kk][d] = fmaf(h, Mv[d], P[kk][d]);
        }
      }
    }
}

template <int KC, int M>
__global__ void __launch_bounds__(256) k_descriptor(PathArgs a) {
    constexpr int D = Moments<M>::D;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = t >> a.nch_log2;
    const int ch = (int)(t & ((1 << a.nch_log2) - 1));
    if (p >= a.n) return;
    float mu[KC], nef[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        mu[kk] = a.mu[ch * KC + kk];
        nef[kk] = -a.eta[ch * KC + kk] * kLog2e;
    }
    const double4 xi = a.xs[p];
    for (int b = 0; b < a.S; ++b) {
        float P[KC][D];
        accumulate_P<KC, M>(a, xi, p, b, mu, nef, P);
        float* Gp = a.G + p * a.F + (b * a.K + ch * KC) * (M + 1);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
            for (int m = 0; m <= M; ++m) {
                float s = 0.0f;
#pragma unroll
                for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) s += kMult[d] * P[kk][d] * P[kk][d];
                Gp[kk * (M + 1) + m] = (m == 0) ? __builtin_sqrtf(s) : s;
            }
        }
    }
}

template <int KC, int M>
__global__ void __launch_bounds__(256) k_adjoint(PathArgs a) {
    constexpr int D = Moments<M>::D;
    __shared__ double red[6][kBlock / 64];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = t >> a.nch_log2;
    const int nch = 1 << a.nch_log2;
    const int ch = (int)(t & (nch - 1));
    float W6[6] = {0, 0, 0, 0, 0, 0};
    if (p < a.n) {
        float mu[KC], nef[KC], m2eta[KC];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            mu[kk] = a.mu[ch * KC + kk];
            nef[kk] = -a.eta[ch * KC + kk] * kLog2e;
            m2eta[kk] = -2.0f * a.eta[ch * KC + kk];
        }
        const double4 xi = a.xs[p];
        float Fo[3] = {0.0f, 0.0f, 0.0f};
        for (int b = 0; b < a.S; ++b) {
            float P[KC][D];
            accumulate_P<KC, M>(a, xi, p, b, mu, nef, P);
            // P' = 2 T sigma' P in place (sigma' = dE/dS from dE/dG).
            const float* dGp = a.dG + p * a.F + (b * a.K + ch * KC) * (M + 1);
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
                for (int m = 0; m <= M; ++m) {
                    const float gbar = dGp[kk * (M + 1) + m];
                    float sbar;
                    if (m == 0) {
                        float s = 0.0f;
#pragma unroll
                        for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) s += kMult[d] * P[kk][d] * P[kk][d];
                        sbar = s > 0.0f ? 0.5f * gbar * __builtin_amdgcn_rsqf(s) : 0.0f;
                    } else {
                        sbar = gbar;
                    }
#pragma unroll
                    for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) P[kk][d] *= 2.0f * kMult[d] * sbar;
                }
            }
            const int nb = a.cnt[(int64_t)b * a.n + p];
            const int64_t base = (int64_t)b * a.cap * a.n + p;
            for (int c0 = 0; c0 < nb; c0 += kBatchAdj) {
              Pair prs[kBatchAdj];
              load_pairs<kBatchAdj>(a, xi, base, c0, nb, prs);
#pragma unroll
              for (int j = 0; j < kBatchAdj; ++j) {
                const Pair& pr = prs[j];
                if (pr.r2 >= a.rc2) continue;
                const float rinv = __builtin_amdgcn_rsqf(pr.r2);
                const float R = pr.r2 * rinv;
                const float ux = pr.dx * rinv, uy = pr.dy * rinv, uz = pr.dz * rinv;
                const float ang = R * a.half_inv_rc;
                const float fc = 0.5f * __builtin_amdgcn_cosf(ang) + 0.5f;
                const float dfc = -0.5f * a.pi_over_rc * __builtin_amdgcn_sinf(ang);
                float Mv[D];
                monomials<M>(ux, uy, uz, Mv);
                float V[D];
#pragma unroll
                for (int d = 0; d < D; ++d) V[d] = 0.0f;
                float s1 = 0.0f;
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const float tt = R - mu[kk];
                    const float e = __builtin_amdgcn_exp2f(nef[kk] * tt * tt);
                    const float h = e * fc;
                    const float dh = e * fmaf(m2eta[kk] * tt, fc, dfc);
                    float U = 0.0f;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        U = fmaf(P[kk][d], Mv[d], U);
                        V[d] = fmaf(P[kk][d], h, V[d]);
                    }
                    s1 = fmaf(U, dh, s1);
                }
                float Ax, Ay, Az, B;
                moment_adjoint<M>(ux, uy, uz, V, Mv, Ax, Ay, Az, B);
                float gx = s1 * ux + rinv * (Ax - ux * B);
                float gy = s1 * uy + rinv * (Ay - uy * B);
                float gz = s1 * uz + rinv * (Az - uz * B);
                for (int off = 1; off < nch; off <<= 1) {
                    gx += __shfl_xor(gx, off);
                    gy += __shfl_xor(gy, off);
                    gz += __shfl_xor(gz, off);
                }
                if (ch == 0) {
                    Fo[0] += gx;
                    Fo[1] += gy;
                    Fo[2] += gz;
                    const int q = pr.q;
                    unsafeAtomicAdd(&a.Fin[3 * (int64_t)q + 0], -gx);
                    unsafeAtomicAdd(&a.Fin[3 * (int64_t)q + 1], -gy);
                    unsafeAtomicAdd(&a.Fin[3 * (int64_t)q + 2], -gz);
                    W6[0] -= pr.dx * gx;
                    W6[1] -= pr.dy * gy;
                    W6[2] -= pr.dz * gz;
                    W6[3] -= 0.5f * (pr.dx * gy + pr.dy * gx);
                    W6[4] -= 0.5f * (pr.dx * gz + pr.dz * gx);
                    W6[5] -= 0.5f * (pr.dy * gz + pr.dz * gy);
                }
              }
            }
        }
        if (ch == 0) {
            a.Fown[3 * p + 0] = Fo[0];
            a.Fown[3 * p + 1] = Fo[1];
            a.Fown[3 * p + 2] = Fo[2];
        }
    }
    // Block reduction of the virial partials in FP64.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double v = (double)W6[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[j][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[threadIdx.x][w];
        a.vir[(int64_t)blockIdx.x * 6 + threadIdx.x] = s;
    }
}

template <int KC>
using KernelFn = void (*)(PathArgs);

template <int KC>
KernelFn<KC> pick_desc(int M) {
    switch (M) {
        case 0: return k_descriptor<KC, 0>;
        case 1: return k_descriptor<KC, 1>;
        case 2: return k_descriptor<KC, 2>;
        default: return k_descriptor<KC, 3>;
    }
}
template <int KC>
KernelFn<KC> pick_adj(int M) {
    switch (M) {
        case 0: return k_adjoint<KC, 0>;
        case 1: return k_adjoint<KC, 1>;
        case 2: return k_adjoint<KC, 2>;
        default: return k_adjoint<KC, 3>;
    }
}

void (*select_kernel(int kc, int M, bool adjoint))(PathArgs) {
    switch (kc) {
        case 4: return adjoint ? pick_adj<4>(M) : pick_desc<4>(M);
        case 6: return adjoint ? pick_adj<6>(M) : pick_desc<6>(M);
        default: return adjoint ? pick_adj<8>(M) : pick_desc<8>(M);
    }
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
    for (int q = 0; q < 3; ++q) a.L[q] = nl->box[q];
    a.xs = nl->xs;
    a.nbr = nl->nbr;
    a.img = nl->img;
    a.cnt = nl->cnt;
    a.mu = m->mu;
    a.eta = m->eta;
    return a;
}

unsigned path_grid(const tmd_model* m, const tmd_nlist* nl) {
    const int64_t threads = nl->n * (m->K / m->kc);
    return (unsigned)((threads + kBlock - 1) / kBlock);
}

}  // namespace

int adjoint_blocks(const tmd_model* m, const tmd_nlist* nl) { return (int)path_grid(m, nl); }

tmd_status launch_descriptors(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, float* G) {
    PathArgs a = make_args(m, nl);
    a.G = G;
    auto fn = select_kernel(m->kc, m->M, false);
    {
        ProfScope ps_(ctx, "descriptor");
        fn<<<path_grid(m, nl), kBlock, 0, ctx->stream>>>(a);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_adjoint(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, const float* dG, float* Fown,
                          float* Fin, double* vir_partials, int* nblocks_out) {
    PathArgs a = make_args(m, nl);
    a.dG = dG;
    a.Fown = Fown;
    a.Fin = Fin;
    a.vir = vir_partials;
    const unsigned grid = path_grid(m, nl);
    auto fn = select_kernel(m->kc, m->M, true);
    {
        ProfScope ps_(ctx, "adjoint");
        fn<<<grid, kBlock, 0, ctx->stream>>>(a);
    }
    TMD_HIP(ctx, hipGetLastError());
    *nblocks_out = (int)grid;
    return TMD_OK;
}

}  // namespace tmd
