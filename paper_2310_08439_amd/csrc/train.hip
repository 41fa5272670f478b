// Force-matching training step on a batch of small periodic systems.
//
// Training is not part of the paper's method (its potentials were fitted
// elsewhere); it fits the per-element MLP to energy and force labels.  The
// batch's configurations are fixed, so everything that depends on positions
// only is computed once when the batch is created: the pair vectors D of each
// system's cell-list neighbour table, the descriptors G and the tensors P.
// Each step then runs, on the whole batch at once:
//   1. per-element MLP forward + input gradient (FP32 MFMA, the inference kernel)
//   2. adjoint per pair (g_c = dE/dD_c, Sec. III.A) into a per-entry buffer
//   3. forces by a deterministic gather F_i = sum_c (g_c - g_mirror(c)), where
//      mirror(c) is the entry of the neighbour's row pointing back at i
//   4. loss terms in FP64 and the seeds e_i = dL/dE_i, r_i = dL/dF_i
//   5. descriptor tangent w_i = d/de G_i(x + e r): forward mode through the
//      descriptor, P_t = sum_c h' R_t M + h M_t, S_t = 2 T P P_t
//   6. second-order MLP pass per tile of atoms (primal + tangent forward,
//      reverse through both) giving per-tile weight-gradient partials
//   7. fixed-order reduction of the partials, then Adam or SGD on the master
//      weights and regeneration of the MLP operand copies.
// Every reduction has a fixed order, so a step is bitwise reproducible.
#include "tmd_internal.h"
#include "tensor_ops.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

struct tmd_batch {
    tmd_context* ctx = nullptr;
    int B = 0;
    int64_t N = 0;
    int S = 0, K = 0, M = 0, D = 0, F = 0, kc = 0, cap = 0;
    // network shape the per-step buffers were sized for (padded widths) and
    // the model's own radial count and feature count (batch reads)
    int H = 0, L = 0, Kabi = 0, Fabi = 0;
    int64_t P_int = 0;
    double rcut = 0.0;
    std::vector<float> mu, eta;  // descriptor parameters the batch was prepared with
    std::vector<int64_t> sys_off_h;
    tmd::SpeciesGroups groups;
    // device
    int64_t* sys_off = nullptr;  // [B+1]
    int32_t* sys_of = nullptr;   // [N]
    int32_t* species = nullptr;  // [N]
    int32_t* sp_idx = nullptr;   // [N] atoms grouped by species
    double* E_label = nullptr;   // [B]
    float* F_label = nullptr;    // [N][3]
    float4* tab = nullptr;       // [N][S][cap] (Dx, Dy, Dz, neighbour index bits)
    int32_t* cnt = nullptr;      // [N][S]
    int32_t* mirror = nullptr;   // [N][S][cap]
    float* G = nullptr;          // [N][F]
    float* P = nullptr;          // [S][K][D][N]
    // per-step buffers
    float* Ei = nullptr;         // [N]
    float* dG = nullptr;         // [N][F]
    float4* g = nullptr;         // [N][S][cap]
    float* Fp = nullptr;         // [N][3]
    float* r = nullptr;          // [N][3]
    float* e = nullptr;          // [N]
    float* w = nullptr;          // [N][F]
    double* sysE = nullptr;      // [B]
    double* sysF = nullptr;      // [B]
    double* loss = nullptr;      // [4]
    float* partial = nullptr;    // [tiles][P_int]
    float* grad = nullptr;       // [S][P_int], the gradient in the padded layout
    int32_t* flag = nullptr;     // [1] set when an entry has no mirror
    int tileT = 0;               // atoms per second-order tile
    int tileQC = 0;              // weight columns per LDS block of the second-order pass
    int tileR = 0;               // sub-tiles of tileT atoms per second-order workgroup
    int64_t tiles = 0;
    int64_t tile_off[tmd::kMaxSpecies + 1] = {0};
};

namespace tmd {
namespace {

using namespace ops;

// ---------------------------------------------------------------- batch set-up

// Copy one system's list (sorted numbering of its cell list) into the batch's
// pair table in batch numbering, with D = (x_j - x_i) + n L evaluated in FP64
// on the wrapped positions and rounded to FP32 as in the inference path.
__global__ void k_pair_rows(int64_t n, int S, int cap_nl, int cap, int64_t off, double Lx, double Ly, double Lz,
                            const int32_t* __restrict__ perm, const double4* __restrict__ xs,
                            const int32_t* __restrict__ nbr, const int32_t* __restrict__ img,
                            const int32_t* __restrict__ cnt, float4* __restrict__ tab, int32_t* __restrict__ tcnt,
                            int32_t* __restrict__ flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t a = off + perm[p];
    const double4 xi = xs[p];
    for (int b = 0; b < S; ++b) {
        const int c_n = cnt[(int64_t)b * n + p];
        if (c_n > cap) {
            atomicOr(flag, 2);
            tcnt[a * S + b] = 0;
            continue;
        }
        tcnt[a * S + b] = c_n;
        const int64_t src = (p * S + b) * cap_nl, dst = (a * S + b) * cap;
        for (int c = 0; c < c_n; ++c) {
            const int q = nbr[src + c];
            int nx, ny, nz;
            unpack_img(img[src + c], nx, ny, nz);
            const double4 xj = xs[q];
            float4 t;
            t.x = (float)((xj.x - xi.x) + (double)nx * Lx);
            t.y = (float)((xj.y - xi.y) + (double)ny * Ly);
            t.z = (float)((xj.z - xi.z) + (double)nz * Lz);
            t.w = __int_as_float((int)(off + perm[q]));
            tab[dst + c] = t;
        }
    }
}

// mirror[(a,b,c)] = the entry of row (j, species(a)) that points back at a
// with the opposite pair vector (exactly -D: both come from the same FP64
// subtraction with swapped operands).
__global__ void k_mirror(int64_t N, int S, int cap, const float4* __restrict__ tab, const int32_t* __restrict__ tcnt,
                         const int32_t* __restrict__ species, int32_t* __restrict__ mirror, int32_t* __restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = t / cap;
    const int c = (int)(t - row * cap);
    if (row >= N * S) return;
    const int64_t a = row / S;
    if (c >= tcnt[row]) return;
    const float4 e = tab[row * cap + c];
    const int64_t j = __float_as_int(e.w);
    const int64_t jrow = j * S + species[a];
    const int n_j = tcnt[jrow];
    int found = -1;
    for (int c2 = 0; c2 < n_j; ++c2) {
        const float4 f = tab[jrow * cap + c2];
        if (__float_as_int(f.w) == (int)a && f.x == -e.x && f.y == -e.y && f.z == -e.z) {
            found = c2;
            break;
        }
    }
    if (found < 0) {
        atomicOr(flag, 1);
        mirror[row * cap + c] = (int32_t)(row * cap + c);  // self: contributes g - g = 0
    } else {
        mirror[row * cap + c] = (int32_t)(jrow * cap + found);
    }
}

struct PtArgs {
    int64_t N;
    int S, K, F, cap, nch_log2;
    float rc2, half_inv_rc, pi_over_rc;
    const float4* tab;
    const int32_t* cnt;
    const float* mu;
    const float* eta;
    float* G;
    float* P;
    const float* dG;
    float4* g;
    const float* r;
    float* w;
};

struct PairGeo {
    float dx, dy, dz, rinv, R, ux, uy, uz;
};

__device__ __forceinline__ bool pair_geo(const float4& e, float rc2, PairGeo& p) {
    p.dx = e.x;
    p.dy = e.y;
    p.dz = e.z;
    const float r2 = p.dx * p.dx + p.dy * p.dy + p.dz * p.dz;
    if (r2 >= rc2) return false;
    p.rinv = __builtin_amdgcn_rsqf(r2);
    p.R = r2 * p.rinv;
    p.ux = p.dx * p.rinv;
    p.uy = p.dy * p.rinv;
    p.uz = p.dz * p.rinv;
    return true;
}

// P tile of (atom a, species b, this thread's chunk) into P; also G and the
// element-major copy of P.
template <int KC, int M>
__global__ void __launch_bounds__(256) k_pt_forward(PtArgs a) {
    constexpr int D = Moments<M>::D;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t >> a.nch_log2;
    const int ch = (int)(t & ((1 << a.nch_log2) - 1));
    if (i >= a.N) return;
    float mu[KC], nef[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        mu[kk] = a.mu[ch * KC + kk];
        nef[kk] = -a.eta[ch * KC + kk] * kLog2e;
    }
    for (int b = 0; b < a.S; ++b) {
        float P[KC][D];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
#pragma unroll
            for (int d = 0; d < D; ++d) P[kk][d] = 0.0f;
        const int64_t row = (i * a.S + b) * a.cap;
        const int nb = a.cnt[i * a.S + b];
        for (int c = 0; c < nb; ++c) {
            PairGeo p;
            if (!pair_geo(a.tab[row + c], a.rc2, p)) continue;
            const float fc = 0.5f * __builtin_amdgcn_cosf(p.R * a.half_inv_rc) + 0.5f;
            float Mv[D];
            monomials<M>(p.ux, p.uy, p.uz, Mv);
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const float tt = p.R - mu[kk];
                const float h = __builtin_amdgcn_exp2f(nef[kk] * tt * tt) * fc;
#pragma unroll
                for (int d = 0; d < D; ++d) P[kk][d] = fmaf(h, Mv[d], P[kk][d]);
            }
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const int k = ch * KC + kk;
#pragma unroll
            for (int d = 0; d < D; ++d) a.P[((int64_t)(b * a.K + k) * D + d) * a.N + i] = P[kk][d];
#pragma unroll
            for (int m = 0; m <= M; ++m) {
                float s = 0.0f;
#pragma unroll
                for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) s += kMult[d] * P[kk][d] * P[kk][d];
                // m = 0 has the single component d = 0: sqrt(S) = |P_k0| exactly
                a.G[i * a.F + (b * a.K + k) * (M + 1) + m] = (m == 0) ? fabsf(P[kk][0]) : s;
            }
        }
    }
}

template <int KC, int D>
__device__ __forceinline__ void load_P(const PtArgs& a, int64_t i, int b, int ch, float (&P)[KC][D]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
        for (int d = 0; d < D; ++d) P[kk][d] = a.P[((int64_t)(b * a.K + ch * KC + kk) * D + d) * a.N + i];
}

// Per-entry g = dE_i/dD_c (the adjoint chain of Sec. III.A); chunk lanes of
// an atom are adjacent and combine their partial sums with shuffles.
template <int KC, int M>
__global__ void __launch_bounds__(256) k_pt_adjoint(PtArgs a) {
    constexpr int D = Moments<M>::D;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t >> a.nch_log2;
    const int nch = 1 << a.nch_log2;
    const int ch = (int)(t & (nch - 1));
    if (i >= a.N) return;
    float mu[KC], nef[KC], m2eta[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        mu[kk] = a.mu[ch * KC + kk];
        nef[kk] = -a.eta[ch * KC + kk] * kLog2e;
        m2eta[kk] = -2.0f * a.eta[ch * KC + kk];
    }
    for (int b = 0; b < a.S; ++b) {
        float P[KC][D];
        load_P<KC, D>(a, i, b, ch, P);
        const float* dGp = a.dG + i * a.F + (b * a.K + ch * KC) * (M + 1);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
            for (int m = 0; m <= M; ++m) {
                const float gbar = dGp[kk * (M + 1) + m];
                if (m == 0) {
                    // G = sqrt(P_k0^2) = |P_k0|, so P'_k0 = G' sign(P_k0) (0 where P_k0 = 0);
                    // no reciprocal square root of a possibly denormal S
                    const float pk = P[kk][0];
                    P[kk][0] = pk > 0.0f ? gbar : (pk < 0.0f ? -gbar : 0.0f);
                } else {
#pragma unroll
                    for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) P[kk][d] *= 2.0f * kMult[d] * gbar;
                }
            }
        }
        const int64_t row = (i * a.S + b) * a.cap;
        const int nb = a.cnt[i * a.S + b];
        for (int c = 0; c < nb; ++c) {
            PairGeo p;
            float gx = 0.0f, gy = 0.0f, gz = 0.0f;
            if (pair_geo(a.tab[row + c], a.rc2, p)) {
                const float ang = p.R * a.half_inv_rc;
                const float fc = 0.5f * __builtin_amdgcn_cosf(ang) + 0.5f;
                const float dfc = -0.5f * a.pi_over_rc * __builtin_amdgcn_sinf(ang);
                float Mv[D], V[D];
                monomials<M>(p.ux, p.uy, p.uz, Mv);
#pragma unroll
                for (int d = 0; d < D; ++d) V[d] = 0.0f;
                float s1 = 0.0f;
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const float tt = p.R - mu[kk];
                    const float ex = __builtin_amdgcn_exp2f(nef[kk] * tt * tt);
                    const float h = ex * fc;
                    const float dh = ex * fmaf(m2eta[kk] * tt, fc, dfc);
                    float U = 0.0f;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        U = fmaf(P[kk][d], Mv[d], U);
                        V[d] = fmaf(P[kk][d], h, V[d]);
                    }
                    s1 = fmaf(U, dh, s1);
                }
                float Ax, Ay, Az, Bm;
                moment_adjoint<M>(p.ux, p.uy, p.uz, V, Mv, Ax, Ay, Az, Bm);
                gx = s1 * p.ux + p.rinv * (Ax - p.ux * Bm);
                gy = s1 * p.uy + p.rinv * (Ay - p.uy * Bm);
                gz = s1 * p.uz + p.rinv * (Az - p.uz * Bm);
            }
            for (int off = 1; off < nch; off <<= 1) {
                gx += __shfl_xor(gx, off);
                gy += __shfl_xor(gy, off);
                gz += __shfl_xor(gz, off);
            }
            if (ch == 0) a.g[row + c] = make_float4(gx, gy, gz, 0.0f);
        }
    }
}

// F_i = sum over i's entries of g_c - g_mirror(c).  Four adjacent lanes per
// atom: lane l sums entries l, l + 4, ... of each row in order, then the
// lanes combine in a fixed butterfly, so the result is reproducible.
constexpr int kForceLanes = 4;
__global__ void k_pt_forces(int64_t N, int S, int cap, const int32_t* __restrict__ tcnt,
                            const int32_t* __restrict__ mirror, const float4* __restrict__ g, float* __restrict__ F) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / kForceLanes;
    const int l = (int)(t % kForceLanes);
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    if (i < N) {
        for (int b = 0; b < S; ++b) {
            const int64_t row = (i * S + b) * cap;
            const int nb = tcnt[i * S + b];
            for (int c = l; c < nb; c += kForceLanes) {
                const float4 u = g[row + c], v = g[mirror[row + c]];
                fx += u.x - v.x;
                fy += u.y - v.y;
                fz += u.z - v.z;
            }
        }
    }
    for (int off = 1; off < kForceLanes; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
    }
    if (i < N && l == 0) {
        F[3 * i + 0] = fx;
        F[3 * i + 1] = fy;
        F[3 * i + 2] = fz;
    }
}

// Per system: E_s = sum of atomic energies and sum |F - Fhat|^2, FP64, fixed
// order (strided per thread, then a tree over the block).
__global__ void __launch_bounds__(256) k_loss_sys(const int64_t* __restrict__ sys_off, const float* __restrict__ Ei,
                                                  const float* __restrict__ F, const float* __restrict__ Fl,
                                                  double* __restrict__ sysE, double* __restrict__ sysF) {
    __shared__ double se[256], sf[256];
    const int s = blockIdx.x, t = threadIdx.x;
    const int64_t lo = sys_off[s], hi = sys_off[s + 1];
    double e = 0.0, f = 0.0;
    for (int64_t i = lo + t; i < hi; i += 256) {
        e += (double)Ei[i];
        for (int x = 0; x < 3; ++x) {
            const double d = (double)F[3 * i + x] - (double)Fl[3 * i + x];
            f += d * d;
        }
    }
    se[t] = e;
    sf[t] = f;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            se[t] += se[t + w];
            sf[t] += sf[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        sysE[s] = se[0];
        sysF[s] = sf[0];
    }
}

// Loss terms (Neumaier over systems in order) and the per-system energy seed.
// One workgroup of 256: the threads form the terms of 256 systems at a time,
// thread 0 adds them in system order.
__global__ void __launch_bounds__(256) k_loss_total(int B, int64_t N, double lambda,
                                                    const int64_t* __restrict__ sys_off,
                                                    const double* __restrict__ E_label, const double* __restrict__ sysE,
                                                    const double* __restrict__ sysF, double* __restrict__ loss,
                                                    double* __restrict__ eseed) {
    __shared__ double te[256], tf[256];
    const int tid = threadIdx.x;
    double le = 0.0, ce = 0.0, lf = 0.0, cf = 0.0;
    auto add = [](double& s, double& c, double x) {
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    };
    for (int base = 0; base < B; base += 256) {
        const int s = base + tid;
        if (s < B) {
            const double ns = (double)(sys_off[s + 1] - sys_off[s]);
            const double de = (sysE[s] - E_label[s]) / ns;
            te[tid] = de * de / (double)B;
            tf[tid] = lambda * sysF[s] / (3.0 * (double)N);
            eseed[s] = 2.0 / (double)B * (sysE[s] - E_label[s]) / (ns * ns);
        }
        __syncthreads();
        if (tid == 0)
            for (int k = 0; k < min(256, B - base); ++k) {
                add(le, ce, te[k]);
                add(lf, cf, tf[k]);
            }
        __syncthreads();
    }
    if (tid == 0) {
        loss[1] = le + ce;
        loss[2] = lf + cf;
        loss[0] = loss[1] + loss[2];
    }
}

// r_i = dL/dF_i = 2 lambda/(3N) (F_i - Fhat_i); e_i = seed of i's system.
__global__ void k_residual(int64_t N, float coef, const int32_t* __restrict__ sys_of, const double* __restrict__ eseed,
                           const float* __restrict__ F, const float* __restrict__ Fl, float* __restrict__ r,
                           float* __restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int x = 0; x < 3; ++x) r[3 * i + x] = coef * (F[3 * i + x] - Fl[3 * i + x]);
    e[i] = (float)eseed[sys_of[i]];
}

// Descriptor tangent along r: forward mode through pair geometry, radial
// functions, monomials, P and S.
template <int KC, int M>
__global__ void __launch_bounds__(256) k_pt_tangent(PtArgs a) {
    constexpr int D = Moments<M>::D;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t >> a.nch_log2;
    const int ch = (int)(t & ((1 << a.nch_log2) - 1));
    if (i >= a.N) return;
    float mu[KC], nef[KC], m2eta[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        mu[kk] = a.mu[ch * KC + kk];
        nef[kk] = -a.eta[ch * KC + kk] * kLog2e;
        m2eta[kk] = -2.0f * a.eta[ch * KC + kk];
    }
    const float rix = a.r[3 * i], riy = a.r[3 * i + 1], riz = a.r[3 * i + 2];
    for (int b = 0; b < a.S; ++b) {
        float Pt[KC][D];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
#pragma unroll
            for (int d = 0; d < D; ++d) Pt[kk][d] = 0.0f;
        const int64_t row = (i * a.S + b) * a.cap;
        const int nb = a.cnt[i * a.S + b];
        for (int c = 0; c < nb; ++c) {
            const float4 ent = a.tab[row + c];
            PairGeo p;
            if (!pair_geo(ent, a.rc2, p)) continue;
            const int64_t j = __float_as_int(ent.w);
            const float tx = a.r[3 * j] - rix, ty = a.r[3 * j + 1] - riy, tz = a.r[3 * j + 2] - riz;
            const float Rt = p.ux * tx + p.uy * ty + p.uz * tz;
            const float utx = (tx - p.ux * Rt) * p.rinv, uty = (ty - p.uy * Rt) * p.rinv,
                        utz = (tz - p.uz * Rt) * p.rinv;
            const float ang = p.R * a.half_inv_rc;
            const float fc = 0.5f * __builtin_amdgcn_cosf(ang) + 0.5f;
            const float dfc = -0.5f * a.pi_over_rc * __builtin_amdgcn_sinf(ang);
            float Mv[D], Mt[D];
            monomials<M>(p.ux, p.uy, p.uz, Mv);
            monomial_tangent<M>(Mv, p.ux, p.uy, p.uz, utx, uty, utz, Mt);
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const float tt = p.R - mu[kk];
                const float ex = __builtin_amdgcn_exp2f(nef[kk] * tt * tt);
                const float h = ex * fc;
                const float dhR = ex * fmaf(m2eta[kk] * tt, fc, dfc) * Rt;
#pragma unroll
                for (int d = 0; d < D; ++d) Pt[kk][d] = fmaf(dhR, Mv[d], fmaf(h, Mt[d], Pt[kk][d]));
            }
        }
        float P[KC][D];
        load_P<KC, D>(a, i, b, ch, P);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const int k = ch * KC + kk;
#pragma unroll
            for (int m = 0; m <= M; ++m) {
                float st = 0.0f;
#pragma unroll
                for (int d = kOrderStart[m]; d < kOrderStart[m + 1]; ++d) st += 2.0f * kMult[d] * P[kk][d] * Pt[kk][d];
                // m = 0: G = |P_k0|, so its tangent is sign(P_k0) times that of P_k0
                float wv = st;
                if (m == 0) wv = P[kk][0] > 0.0f ? Pt[kk][0] : (P[kk][0] < 0.0f ? -Pt[kk][0] : 0.0f);
                a.w[i * a.F + (b * a.K + k) * (M + 1) + m] = wv;
            }
        }
    }
}

// ---------------------------------------------------------------- second-order MLP pass

struct MlpTrainArgs {
    int S, F, L, H, act, T, QC, R, P;
    int64_t sp_off[kMaxSpecies + 1];
    int64_t tile_off[kMaxSpecies + 1];
    const int32_t* sp_idx;
    const float* G;
    const float* w;
    const float* e;
    const float* params;  // [S][P]
    float* partial;       // [tiles][P]
};

__device__ __forceinline__ float sig(int act, float z) {
    if (act == TMD_ACT_SQUAREPLUS) return 0.5f * (z + sqrtf(z * z + 4.0f));
    return tanhf(z);
}
__device__ __forceinline__ float dsig(int act, float z) {
    if (act == TMD_ACT_SQUAREPLUS) return 0.5f * (1.0f + z / sqrtf(z * z + 4.0f));
    const float t = tanhf(z);
    return 1.0f - t * t;
}
__device__ __forceinline__ float d2sig(int act, float z) {
    if (act == TMD_ACT_SQUAREPLUS) {
        const float q = z * z + 4.0f;
        return 2.0f / (q * sqrtf(q));
    }
    const float t = tanhf(z);
    return -2.0f * t * (1.0f - t * t);
}

// One workgroup per tile of up to T atoms of one species; activations of the
// tile live in LDS as [width][Tp] with the odd row stride Tp = T | 1, so that
// lanes walking the width at a fixed atom hit distinct banks.  The weights of
// a layer pass through LDS in blocks of QC input columns, [H][QC + 1].
// Primal z_l = W_l a_{l-1} + b_l, a_l = s(z_l); tangent zt_l = W_l at_{l-1},
// at_l = s'(z_l) zt_l, from a_0 = G, at_0 = w.  Reverse mode of
// J = e E - w_out . at_L through both graphs:
//   ztbar_l = s'(z_l) atbar_l,  zbar_l = s'(z_l) abar_l + s''(z_l) zt_l atbar_l,
//   dW_l += zbar_l a_{l-1}^T + ztbar_l at_{l-1}^T,  db_l += zbar_l,
//   abar_{l-1} = W_l^T zbar_l,  atbar_{l-1} = W_l^T ztbar_l.
template <int T, int NR>
__global__ void __launch_bounds__(256) k_mlp_second(MlpTrainArgs a) {
    extern __shared__ float lds[];
    constexpr int Tp = T | 1;
    const int H = a.H, F = a.F, L = a.L, QC = a.QC;
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    int s = 0;
    for (int q = 0; q < a.S; ++q)
        if (tile >= a.tile_off[q] && tile < a.tile_off[q + 1]) s = q;
    const int64_t first0 = a.sp_off[s] + (tile - a.tile_off[s]) * (int64_t)T * a.R;
    float* X0 = lds;                      // [F][Tp]
    float* X0t = X0 + F * Tp;             // [F][Tp]
    float* Z = X0t + F * Tp;              // [L][H][Tp]
    float* A = Z + L * H * Tp;
    float* Zt = A + L * H * Tp;
    float* At = Zt + L * H * Tp;
    float* Ba = At + L * H * Tp;          // [H][Tp]
    float* Bat = Ba + H * Tp;
    float* Cz = Bat + H * Tp;
    float* Czt = Cz + H * Tp;
    float* Ws = Czt + H * Tp;             // [H][QC + 1]
    float* Es = Ws + H * (QC + 1);        // [T] energy seeds, 0 past the tile's last atom
    constexpr int G = 256 / T;            // rows of a [width][T] array covered by one pass of the workgroup
    const int tcol = tid % T, row0 = tid / T;  // this thread's column and first row
    const float* p = a.params + (int64_t)s * a.P;
    float* gp = a.partial + tile * a.P;
    // Ws[o][c] = W[o][q0 + c] for c < qn; the caller synchronises.
    auto stage = [&](const float* W, int wi, int q0, int qn) {
        for (int idx = tid; idx < H * qn; idx += blockDim.x) {
            const int o = idx / qn, c = idx - o * qn;
            Ws[o * (QC + 1) + c] = W[(int64_t)o * wi + q0 + c];
        }
    };

    // The workgroup's tile is R sub-tiles of T atoms, taken in order; each
    // adds its weight-gradient terms to the tile's partial row.
    for (int r = 0; r < a.R; ++r) {
        const int64_t first = first0 + (int64_t)r * T;
        if (first >= a.sp_off[s + 1]) break;  // the same for the whole workgroup
        const int nt = (int)min((int64_t)T, a.sp_off[s + 1] - first);
        auto put = [&](int64_t k, float v) { gp[k] = r == 0 ? v : gp[k] + v; };
        // Past the tile's last atom the inputs, tangents and seeds are zero, so
        // the cotangents Cz, Czt of those columns are exactly zero and the sums
        // over the tile can run over all T columns.
        if (tid < T) Es[tid] = tid < nt ? a.e[a.sp_idx[first + tid]] : 0.0f;
        for (int idx = tid; idx < F * T; idx += blockDim.x) {
            const int q = idx / T, t = idx - q * T;
            float g = 0.0f, wt = 0.0f;
            if (t < nt) {
                const int64_t atom = a.sp_idx[first + t];
                g = a.G[atom * F + q];
                wt = a.w[atom * F + q];
            }
            X0[q * Tp + t] = g;
            X0t[q * Tp + t] = wt;
        }
        // forward: primal and tangent, accumulated over the weight blocks in Z, Zt
        int off = 0;
        int offW[TMD_MAX_HIDDEN], offb[TMD_MAX_HIDDEN];
        for (int l = 0; l < L; ++l) {
            const int wi = (l == 0) ? F : H;
            offW[l] = off;
            off += H * wi;
            offb[l] = off;
            off += H;
            const float* in = (l == 0) ? X0 : A + (l - 1) * H * Tp;
            const float* int_ = (l == 0) ? X0t : At + (l - 1) * H * Tp;
            float* Zl = Z + l * H * Tp;
            float* Ztl = Zt + l * H * Tp;
            for (int q0 = 0; q0 < wi; q0 += QC) {
                const int qn = min(QC, wi - q0);
                const bool last = q0 + qn == wi;
                stage(p + offW[l], wi, q0, qn);
                __syncthreads();
                // thread (tcol, row0) owns rows row0, row0 + G, row0 + 2G, ... of column tcol;
                // NR rows at a time share the loads of the inputs
                for (int ob = row0; ob < H; ob += NR * G) {
                    float z[NR], zt[NR];
#pragma unroll
                    for (int k = 0; k < NR; ++k) {
                        const int o = min(ob + k * G, H - 1);
                        z[k] = q0 == 0 ? p[offb[l] + o] : Zl[o * Tp + tcol];
                        zt[k] = q0 == 0 ? 0.0f : Ztl[o * Tp + tcol];
                    }
                    const float* ip = in + q0 * Tp + tcol;
                    const float* itp = int_ + q0 * Tp + tcol;
#pragma unroll 2
                    for (int c = 0; c < qn; ++c) {
                        const float x = ip[c * Tp], xt = itp[c * Tp];
#pragma unroll
                        for (int k = 0; k < NR; ++k) {
                            const float wv = Ws[min(ob + k * G, H - 1) * (QC + 1) + c];
                            z[k] = fmaf(wv, x, z[k]);
                            zt[k] = fmaf(wv, xt, zt[k]);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < NR; ++k) {
                        const int o = ob + k * G;
                        if (o < H) {
                            Zl[o * Tp + tcol] = z[k];
                            Ztl[o * Tp + tcol] = zt[k];
                            if (last) {
                                A[(l * H + o) * Tp + tcol] = sig(a.act, z[k]);
                                At[(l * H + o) * Tp + tcol] = dsig(a.act, z[k]) * zt[k];
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        const int offWo = off, offbo = off + H;
        // output layer: E = w_out . a_L + b_out, q = w_out . at_L
        for (int idx = tid; idx < H * T; idx += blockDim.x) {
            const int o = idx / T, t = idx - o * T;
            const bool live = t < nt;
            Ba[o * Tp + t] = live ? Es[t] * p[offWo + o] : 0.0f;
            Bat[o * Tp + t] = live ? -p[offWo + o] : 0.0f;
        }
        for (int o = tid; o < H; o += blockDim.x) {
            float gw = 0.0f;
#pragma unroll
            for (int t = 0; t < T; ++t) gw += Es[t] * A[((L - 1) * H + o) * Tp + t] - At[((L - 1) * H + o) * Tp + t];
            put(offWo + o, gw);
        }
        if (tid == 0) {
            float gb = 0.0f;
#pragma unroll
            for (int t = 0; t < T; ++t) gb += Es[t];
            put(offbo, gb);
        }
        __syncthreads();
        for (int l = L - 1; l >= 0; --l) {
            const int wi = (l == 0) ? F : H;
            for (int idx = tid; idx < H * T; idx += blockDim.x) {
                const int o = idx / T, t = idx - o * T;
                const int at = o * Tp + t;
                const float z = Z[l * H * Tp + at];
                const float d1 = dsig(a.act, z), d2 = d2sig(a.act, z);
                Czt[at] = d1 * Bat[at];
                Cz[at] = d1 * Ba[at] + d2 * Zt[l * H * Tp + at] * Bat[at];
            }
            __syncthreads();
            const float* in = (l == 0) ? X0 : A + (l - 1) * H * Tp;
            const float* int_ = (l == 0) ? X0t : At + (l - 1) * H * Tp;
            if (256 % wi == 0) {
                // each thread keeps one input row q for all its rows o
                const int q = tid % wi;
                float xi[T], xt[T];
#pragma unroll
                for (int u = 0; u < T; ++u) {
                    xi[u] = in[q * Tp + u];
                    xt[u] = int_[q * Tp + u];
                }
                for (int o = tid / wi; o < H; o += 256 / wi) {
                    float gw = 0.0f;
#pragma unroll
                    for (int u = 0; u < T; ++u) gw += Cz[o * Tp + u] * xi[u] + Czt[o * Tp + u] * xt[u];
                    put(offW[l] + o * wi + q, gw);
                }
            } else {
                for (int idx = tid; idx < H * wi; idx += blockDim.x) {
                    const int o = idx / wi, q = idx - o * wi;
                    float gw = 0.0f;
#pragma unroll
                    for (int u = 0; u < T; ++u)
                        gw += Cz[o * Tp + u] * in[q * Tp + u] + Czt[o * Tp + u] * int_[q * Tp + u];
                    put(offW[l] + idx, gw);
                }
            }
            for (int o = tid; o < H; o += blockDim.x) {
                float gb = 0.0f;
#pragma unroll
                for (int t = 0; t < T; ++t) gb += Cz[o * Tp + t];
                put(offb[l] + o, gb);
            }
            if (l > 0) {
                // Ba, Bat = W_l^T (Cz, Czt), one block of input columns at a time
                for (int q0 = 0; q0 < wi; q0 += QC) {
                    const int qn = min(QC, wi - q0);
                    stage(p + offW[l], wi, q0, qn);
                    __syncthreads();
                    // thread (tcol, row0) owns block columns row0, row0 + G, ... of atom tcol;
                    // NR at a time share the loads of Cz, Czt
                    for (int cb = row0; cb < qn; cb += NR * G) {
                        float sa[NR] = {}, st[NR] = {};
#pragma unroll 2
                        for (int o = 0; o < H; ++o) {
                            const float cz = Cz[o * Tp + tcol], czt = Czt[o * Tp + tcol];
#pragma unroll
                            for (int k = 0; k < NR; ++k) {
                                const float wv = Ws[o * (QC + 1) + min(cb + k * G, qn - 1)];
                                sa[k] = fmaf(wv, cz, sa[k]);
                                st[k] = fmaf(wv, czt, st[k]);
                            }
                        }
#pragma unroll
                        for (int k = 0; k < NR; ++k) {
                            const int c = cb + k * G;
                            if (c < qn) {
                                Ba[(q0 + c) * Tp + tcol] = sa[k];
                                Bat[(q0 + c) * Tp + tcol] = st[k];
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            __syncthreads();
        }
    }
}

// Fixed-order reduction of the per-tile partials of each species, in two
// passes so that it spreads over the chip: the tiles of species s form chunks
// of kGradChunk consecutive tiles; pass one sums each chunk in tile order and
// leaves the sum in the chunk's first row, pass two sums the chunks in order.
constexpr int kGradChunk = 32;

struct GradReduceArgs {
    int S, P;
    int64_t tile_off[kMaxSpecies + 1];   // tiles of species s: [tile_off[s], tile_off[s + 1])
    int64_t chunk_off[kMaxSpecies + 1];  // chunks of species s: [chunk_off[s], chunk_off[s + 1])
    float* partial;                      // [tiles][P]
    float* grad;                         // [S][P]
};

// One thread per (chunk, parameter); workgroup x = chunk * pb + (parameter / 256)
// with pb = ceil(P / 256).
__global__ void __launch_bounds__(256) k_grad_chunks(GradReduceArgs a, int pb) {
    const int64_t c = blockIdx.x / pb;
    const int q = (int)(blockIdx.x - c * pb) * 256 + threadIdx.x;
    if (q >= a.P) return;
    int s = 0;
    for (int k = 0; k < a.S; ++k)
        if (c >= a.chunk_off[k] && c < a.chunk_off[k + 1]) s = k;
    const int64_t lo = a.tile_off[s] + (c - a.chunk_off[s]) * kGradChunk;
    const int64_t hi = min(lo + kGradChunk, a.tile_off[s + 1]);
    float acc = 0.0f;
#pragma unroll 8
    for (int64_t tl = lo; tl < hi; ++tl) acc += a.partial[tl * a.P + q];
    a.partial[lo * a.P + q] = acc;
}

// grad[s][q] = sum over the chunks of species s, in chunk order.
__global__ void k_grad_reduce(GradReduceArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.S * a.P) return;
    const int s = (int)(t / a.P), q = (int)(t - (int64_t)s * a.P);
    float acc = 0.0f;
#pragma unroll 8
    for (int64_t lo = a.tile_off[s]; lo < a.tile_off[s + 1]; lo += kGradChunk) acc += a.partial[lo * a.P + q];
    a.grad[t] = acc;
}

// Adam (or SGD when beta1 < 0) on the master weights.
__global__ void k_optimizer(int64_t n, int adam, float lr, float b1, float b2, float eps, float c1, float c2,
                            const float* __restrict__ g, float* __restrict__ theta, float* __restrict__ m,
                            float* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!adam) {
        theta[i] -= lr * g[i];
        return;
    }
    const float mi = b1 * m[i] + (1.0f - b1) * g[i];
    const float vi = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct UnpackArgs {
    int S, L, H, Fpad;
    int64_t P, P_int, wstride;
    int64_t w_off[TMD_MAX_HIDDEN], wt_off[TMD_MAX_HIDDEN];
    ParamMap pm;
    const float* params;
    float* params_int;  // null when the model is not padded
    float* w32;
    __hip_bfloat16* wbf;
    float* bias;
    float* wout;
    float* bout;
};

// One thread per master parameter (ABI layout): write it to every operand
// copy and to the padded master copy.  Padded entries are never written and
// stay zero.
__global__ void k_unpack(UnpackArgs u) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)u.S * u.P) return;
    const int s = (int)(t / u.P);
    const int64_t q = t - (int64_t)s * u.P;
    const float v = u.params[t];
    int l, o, c, kind;
    const int64_t qi = u.pm.map(q, l, o, c, kind);
    if (u.params_int) u.params_int[(int64_t)s * u.P_int + qi] = v;
    if (kind == 0) {
        float* ws = u.w32 + s * u.wstride;
        __hip_bfloat16* wb = u.wbf + s * u.wstride;
        const int in_pad = (l == 0) ? u.Fpad : u.H;
        ws[u.w_off[l] + (int64_t)o * in_pad + c] = v;
        ws[u.wt_off[l] + (int64_t)c * u.H + o] = v;
        wb[u.w_off[l] + (int64_t)o * in_pad + c] = __float2bfloat16(v);
        wb[u.wt_off[l] + (int64_t)c * u.H + o] = __float2bfloat16(v);
    } else if (kind == 1) {
        u.bias[((int64_t)s * u.L + l) * u.H + o] = v;
    } else if (kind == 2) {
        u.wout[(int64_t)s * u.H + o] = v;
    } else {
        u.bout[s] = v;
    }
}

// Gradient of a padded model back to the ABI layout: out[s][q] = in[s][map(q)].
__global__ void k_grad_compact(int S, int64_t P, int64_t P_int, ParamMap pm, const float* __restrict__ in,
                               float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)S * P) return;
    const int s = (int)(t / P);
    int l, o, c, kind;
    const int64_t qi = pm.map(t - (int64_t)s * P, l, o, c, kind);
    out[t] = in[(int64_t)s * P_int + qi];
}

using PtFn = void (*)(PtArgs);

#define TMD_PICK(NAME, KERNEL)                                    \
    PtFn NAME(int kc, int M) {                                    \
        switch (kc * 10 + M) {                                    \
            case 20: return KERNEL<2, 0>;                         \
            case 21: return KERNEL<2, 1>;                         \
            case 22: return KERNEL<2, 2>;                         \
            case 23: return KERNEL<2, 3>;                         \
            case 40: return KERNEL<4, 0>;                         \
            case 41: return KERNEL<4, 1>;                         \
            case 42: return KERNEL<4, 2>;                         \
            case 43: return KERNEL<4, 3>;                         \
            case 60: return KERNEL<6, 0>;                         \
            case 61: return KERNEL<6, 1>;                         \
            case 62: return KERNEL<6, 2>;                         \
            case 63: return KERNEL<6, 3>;                         \
            case 80: return KERNEL<8, 0>;                         \
            case 81: return KERNEL<8, 1>;                         \
            case 82: return KERNEL<8, 2>;                         \
            default: return KERNEL<8, 3>;                         \
        }                                                         \
    }
TMD_PICK(pick_forward, k_pt_forward)
TMD_PICK(pick_adjoint, k_pt_adjoint)
TMD_PICK(pick_tangent, k_pt_tangent)
#undef TMD_PICK

unsigned blocks_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

// Radial functions per thread of the pair-table kernels: the model's chunk,
// halved (8 -> 4 -> 2) while the batch would give fewer than 1024 threads per
// compute unit.  P is stored by radial index, so any chunk reads it.
int batch_kc(int K, int kc, int64_t N) {
    while (kc % 4 == 0 && N * (K / kc) < (int64_t)256 * 1024 && 2 * K / kc <= 64) kc /= 2;
    return kc;
}

PtArgs pt_args(const tmd_batch* bt) {
    PtArgs a{};
    a.N = bt->N;
    a.S = bt->S;
    a.K = bt->K;
    a.F = bt->F;
    a.cap = bt->cap;
    int nch = bt->K / bt->kc, lg = 0;
    while ((1 << lg) < nch) ++lg;
    a.nch_log2 = lg;
    a.rc2 = (float)(bt->rcut * bt->rcut);
    a.half_inv_rc = (float)(0.5 / bt->rcut);
    a.pi_over_rc = (float)(M_PI / bt->rcut);
    a.tab = bt->tab;
    a.cnt = bt->cnt;
    return a;
}

void batch_free(tmd_batch* b) {
    for (void* p : {(void*)b->sys_off, (void*)b->sys_of, (void*)b->species, (void*)b->sp_idx, (void*)b->E_label,
                    (void*)b->F_label, (void*)b->tab, (void*)b->cnt, (void*)b->mirror, (void*)b->G, (void*)b->P,
                    (void*)b->Ei, (void*)b->dG, (void*)b->g, (void*)b->Fp, (void*)b->r, (void*)b->e, (void*)b->w,
                    (void*)b->sysE, (void*)b->sysF, (void*)b->loss, (void*)b->partial, (void*)b->grad,
                    (void*)b->flag})
        if (p) (void)hipFree(p);
    b->tab = nullptr;
    b->cnt = nullptr;
    b->mirror = nullptr;
}

// LDS bytes of k_mlp_second: activations [width][T | 1], a [H][QC + 1]
// block of weights and the tile's T energy seeds.
size_t mlp2_lds(int F, int H, int L, int T, int QC) {
    return sizeof(float) * ((size_t)(T | 1) * (2 * F + 4 * L * H + 4 * H) + (size_t)H * (QC + 1) + T);
}

// Largest sub-tile of at most 8 atoms, then widest weight block (columns),
// that fit in 64 KB of LDS; false when none does.  (16-atom sub-tiles were
// slower for the 32-64-64-1 network: two workgroups per CU instead of three.)
bool mlp2_shape(int F, int H, int L, int* T, int* QC) {
    for (int t : {8, 4, 2, 1})
        for (int q : {64, 32, 16, 8, 4, 2, 1}) {
            if (mlp2_lds(F, H, L, t, q) <= 64 * 1024) {
                *T = t;
                *QC = q;
                return true;
            }
        }
    return false;
}

}  // namespace
}  // namespace tmd

using namespace tmd;

extern "C" {

tmd_status tmd_batch_create(tmd_context* ctx, const tmd_model* m, int32_t n_systems, const int64_t* sys_off,
                            const double* pos, const int32_t* species, const double* boxes,
                            const double* energy_labels, const float* force_labels, int32_t capacity,
                            tmd_batch** out) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (!m || !sys_off || !pos || !species || !boxes || !energy_labels || !force_labels || !out)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null argument");
    *out = nullptr;
    if (n_systems < 1) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "n_systems must be positive");
    if (sys_off[0] != 0) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "sys_off[0] must be 0");
    int64_t nmax = 0;
    for (int s = 0; s < n_systems; ++s) {
        const int64_t ns = sys_off[s + 1] - sys_off[s];
        if (ns <= 0) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "every system needs at least one atom");
        nmax = std::max(nmax, ns);
        for (int x = 0; x < 3; ++x)
            if (!(boxes[3 * s + x] > 0.0) || !std::isfinite(boxes[3 * s + x]))
                return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "box edges must be positive and finite");
        if (!std::isfinite(energy_labels[s])) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "non-finite energy label");
    }
    const int64_t N = sys_off[n_systems];
    if (N >= ((int64_t)1 << 31) / 8) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "batch too large");
    int tileT = 0, tileQC = 0;
    if (m->F > 1024 || !mlp2_shape(m->F, m->H, m->L, &tileT, &tileQC))
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "model too wide for the training kernels");

    tmd_batch* b = new (std::nothrow) tmd_batch();
    if (!b) return fail(ctx, TMD_ERR_OUT_OF_MEMORY, "host allocation");
    b->ctx = ctx;
    b->B = n_systems;
    b->N = N;
    b->S = m->S;
    b->K = m->K;
    b->M = m->M;
    b->D = m->D;
    b->F = m->F;
    b->H = m->H;
    b->L = m->L;
    b->Kabi = m->Kabi;
    b->Fabi = m->Fabi;
    b->P_int = m->per_species_int;
    b->kc = batch_kc(m->K, m->kc, N);
    b->rcut = m->rcut;
    b->mu.resize(m->K);
    b->eta.resize(m->K);
    b->sys_off_h.assign(sys_off, sys_off + n_systems + 1);

    auto bail = [&](tmd_status st) {
        (void)hipStreamSynchronize(ctx->stream);
        batch_free(b);
        delete b;
        return st;
    };
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 256));
    };
    e = hipMemcpy(b->mu.data(), m->mu, 4 * m->K, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(b->eta.data(), m->eta, 4 * m->K, hipMemcpyDeviceToHost);
    // species on the host: validation and grouping
    std::vector<int32_t> sp_h(N);
    if (e == hipSuccess) e = hipMemcpy(sp_h.data(), species, 4 * N, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "batch upload"));
    std::vector<int32_t> sys_of_h(N), idx_h;
    idx_h.reserve(N);
    for (int s = 0; s < n_systems; ++s)
        for (int64_t i = sys_off[s]; i < sys_off[s + 1]; ++i) sys_of_h[i] = s;
    b->groups.S = m->S;
    for (int s = 0; s < m->S; ++s) {
        b->groups.off[s] = (int64_t)idx_h.size();
        for (int64_t i = 0; i < N; ++i) {
            if (sp_h[i] < 0 || sp_h[i] >= m->S) return bail(fail(ctx, TMD_ERR_INVALID_ARGUMENT, "species out of range"));
            if (sp_h[i] == s) idx_h.push_back((int32_t)i);
        }
    }
    b->groups.off[m->S] = N;

    alloc((void**)&b->sys_off, 8 * (size_t)(n_systems + 1));
    alloc((void**)&b->sys_of, 4 * (size_t)N);
    alloc((void**)&b->species, 4 * (size_t)N);
    alloc((void**)&b->sp_idx, 4 * (size_t)N);
    alloc((void**)&b->E_label, 8 * (size_t)n_systems);
    alloc((void**)&b->F_label, 12 * (size_t)N);
    alloc((void**)&b->cnt, 4 * (size_t)N * m->S);
    alloc((void**)&b->G, 4 * (size_t)N * m->F);
    alloc((void**)&b->P, 4 * (size_t)N * m->S * m->K * m->D);
    alloc((void**)&b->Ei, 4 * (size_t)N);
    alloc((void**)&b->dG, 4 * (size_t)N * m->F);
    alloc((void**)&b->Fp, 12 * (size_t)N);
    alloc((void**)&b->r, 12 * (size_t)N);
    alloc((void**)&b->e, 4 * (size_t)N);
    alloc((void**)&b->w, 4 * (size_t)N * m->F);
    alloc((void**)&b->sysE, 8 * (size_t)n_systems);
    alloc((void**)&b->sysF, 8 * (size_t)n_systems);
    alloc((void**)&b->loss, 8 * 4 + 8 * (size_t)n_systems);
    alloc((void**)&b->grad, 4 * (size_t)m->S * m->per_species_int);
    alloc((void**)&b->flag, 4);
    if (e == hipSuccess) e = hipMemcpy(b->sys_off, sys_off, 8 * (size_t)(n_systems + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->sys_of, sys_of_h.data(), 4 * (size_t)N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->species, sp_h.data(), 4 * (size_t)N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->sp_idx, idx_h.data(), 4 * (size_t)N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->E_label, energy_labels, 8 * (size_t)n_systems, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->F_label, force_labels, 12 * (size_t)N, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "batch allocation"));
    b->groups.idx = b->sp_idx;

    // Pair table: each system's cell list, converted; grown and redone when a
    // row does not fit.
    int cap = std::max(16, capacity > 0 ? capacity : 64);
    for (;;) {
        cap = (cap + 3) / 4 * 4;
        b->cap = cap;
        if (b->tab) (void)hipFree(b->tab);
        b->tab = nullptr;
        alloc((void**)&b->tab, 16 * (size_t)N * m->S * cap);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "pair table allocation"));
        tmd_nlist* nl = nullptr;
        tmd_status st = tmd_nlist_create(ctx, nmax, m->S, cap, &nl);
        if (st != TMD_OK) return bail(st);
        int32_t grow = 0;
        e = hipMemsetAsync(b->flag, 0, 4, ctx->stream);
        if (e != hipSuccess) {
            tmd_nlist_destroy(nl);
            return bail(hip_fail(ctx, e, "pair table"));
        }
        for (int s = 0; s < n_systems && st == TMD_OK; ++s) {
            tmd_system_view v{};
            v.n_atoms = sys_off[s + 1] - sys_off[s];
            v.pos = pos + 3 * sys_off[s];
            v.species = species + sys_off[s];
            for (int x = 0; x < 3; ++x) v.box[x] = boxes[3 * s + x];
            int32_t req = 0;
            st = tmd_build_neighbors(ctx, &v, m->rcut, 0.0, nl, &req);
            if (st == TMD_ERR_CAPACITY) {
                grow = std::max(grow, req);
                st = TMD_OK;
                continue;
            }
            if (st != TMD_OK) break;
            k_pair_rows<<<blocks_for(v.n_atoms), kBlock, 0, ctx->stream>>>(
                v.n_atoms, m->S, nl->cap, cap, sys_off[s], v.box[0], v.box[1], v.box[2], nl->perm, nl->xs, nl->nbr,
                nl->img, nl->cnt, b->tab, b->cnt, b->flag);
            e = hipGetLastError();
            if (e != hipSuccess) break;
            e = hipStreamSynchronize(ctx->stream);  // the list is rebuilt for the next system
            if (e != hipSuccess) break;
        }
        tmd_nlist_destroy(nl);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "pair table"));
        if (st != TMD_OK) return bail(st);
        if (grow > 0) {
            cap = std::max(grow, cap + 4);
            continue;
        }
        break;
    }
    if (N * m->S * (int64_t)b->cap >= ((int64_t)1 << 31))
        return bail(fail(ctx, TMD_ERR_INVALID_ARGUMENT, "pair table larger than 2^31 entries"));
    alloc((void**)&b->mirror, 4 * (size_t)N * m->S * b->cap);
    alloc((void**)&b->g, 16 * (size_t)N * m->S * b->cap);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "pair table allocation"));
    {
        const int64_t entries = N * m->S * b->cap;
        k_mirror<<<blocks_for(entries), kBlock, 0, ctx->stream>>>(N, m->S, b->cap, b->tab, b->cnt, b->species,
                                                                   b->mirror, b->flag);
        PtArgs a = pt_args(b);
        a.mu = m->mu;
        a.eta = m->eta;
        a.G = b->G;
        a.P = b->P;
        pick_forward(b->kc, b->M)<<<blocks_for(N * (b->K / b->kc)), kBlock, 0, ctx->stream>>>(a);
        e = hipGetLastError();
        int32_t flag = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&flag, b->flag, 4, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "batch descriptors"));
        if (flag) return bail(fail(ctx, TMD_ERR_NUMERICAL, "pair table inconsistent (an entry without its mirror)"));
    }
    // second-order tiles
    b->tileT = tileT;
    b->tileQC = tileQC;
    {
        // sub-tiles per workgroup: enough that the grid fills the workgroup
        // slots the LDS allows about once
        const size_t lds = mlp2_lds(m->F, m->H, m->L, tileT, tileQC);
        const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(160 * 1024 / lds)));
        const int64_t slots = (int64_t)ctx->num_cus * per_cu;
        int64_t sub = 0;
        for (int s = 0; s < m->S; ++s) sub += (b->groups.off[s + 1] - b->groups.off[s] + tileT - 1) / tileT;
        b->tileR = (int)std::max<int64_t>(1, (sub + slots - 1) / slots);
    }
    const int64_t tile_atoms_n = (int64_t)b->tileT * b->tileR;
    int64_t tiles = 0;
    for (int s = 0; s < m->S; ++s) {
        b->tile_off[s] = tiles;
        tiles += (b->groups.off[s + 1] - b->groups.off[s] + tile_atoms_n - 1) / tile_atoms_n;
    }
    b->tile_off[m->S] = tiles;
    b->tiles = tiles;
    alloc((void**)&b->partial, 4 * (size_t)std::max<int64_t>(tiles, 1) * m->per_species_int);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "training workspace"));
    *out = b;
    return TMD_OK;
}

void tmd_batch_destroy(tmd_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    batch_free(b);
    delete b;
}

tmd_status tmd_train_step(tmd_context* ctx, tmd_model* m, const tmd_batch* bc, const tmd_train_opts* opts,
                          double* loss, float* grad) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (!m || !bc || !opts || !loss) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null argument");
    tmd_batch* b = const_cast<tmd_batch*>(bc);  // per-step scratch lives in the batch
    if (m->S != b->S || m->K != b->K || m->M != b->M || m->rcut != b->rcut)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "model descriptor shape differs from the batch's");
    // the per-step buffers (second-order tiles, partial and gradient rows) are
    // sized for the network shape of the model the batch was created with
    if (m->H != b->H || m->L != b->L || m->per_species_int != b->P_int)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT,
                    "network shape differs from the one the batch was created for (create a batch for this model)");
    {
        std::vector<float> mu(m->mu_h.begin(), m->mu_h.end()), eta(m->eta_h.begin(), m->eta_h.end());
        if (mu != b->mu || eta != b->eta)
            return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "model radial functions differ from the batch's");
    }
    if (m->tab)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT,
                    "training uses the exact radial functions: drop the table (tmd_model_tabulate(m, 0)) first");
    if (!(opts->lambda >= 0.0) || !(opts->lr >= 0.0) || !std::isfinite(opts->lr))
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "lambda and lr must be non-negative");
    if (opts->optimizer != TMD_OPT_ADAM && opts->optimizer != TMD_OPT_SGD)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "unknown optimizer");
    if (opts->optimizer == TMD_OPT_ADAM && opts->lr > 0.0 &&
        !(opts->beta1 >= 0.0 && opts->beta1 < 1.0 && opts->beta2 >= 0.0 && opts->beta2 < 1.0 && opts->eps > 0.0))
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "Adam needs 0 <= beta < 1 and eps > 0");
    tmd_status st;
    const int64_t N = b->N;
    // 1. energies and input gradients (FP32)
    if ((st = launch_mlp(ctx, m, b->groups, TMD_FP32, b->G, nullptr, b->Ei, b->dG)) != TMD_OK) return st;
    PtArgs a = pt_args(b);
    a.mu = m->mu;
    a.eta = m->eta;
    a.P = b->P;
    a.dG = b->dG;
    a.g = b->g;
    a.r = b->r;
    a.w = b->w;
    const unsigned pt_grid = blocks_for(N * (b->K / b->kc));
    {
        ProfScope ps_(ctx, "train_adjoint");
        pick_adjoint(b->kc, b->M)<<<pt_grid, kBlock, 0, ctx->stream>>>(a);
    }
    {
        ProfScope ps_(ctx, "train_forces");
        k_pt_forces<<<blocks_for(N * kForceLanes), kBlock, 0, ctx->stream>>>(N, b->S, b->cap, b->cnt, b->mirror, b->g, b->Fp);
    }
    // 2. loss and seeds
    {
        ProfScope ps_(ctx, "train_loss");
        double* eseed = b->loss + 4;
        k_loss_sys<<<b->B, 256, 0, ctx->stream>>>(b->sys_off, b->Ei, b->Fp, b->F_label, b->sysE, b->sysF);
        k_loss_total<<<1, 256, 0, ctx->stream>>>(b->B, N, opts->lambda, b->sys_off, b->E_label, b->sysE, b->sysF,
                                                b->loss, eseed);
        k_residual<<<blocks_for(N), kBlock, 0, ctx->stream>>>(N, (float)(2.0 * opts->lambda / (3.0 * (double)N)),
                                                               b->sys_of, eseed, b->Fp, b->F_label, b->r, b->e);
    }
    // 3. descriptor tangent along r
    {
        ProfScope ps_(ctx, "train_tangent");
        pick_tangent(b->kc, b->M)<<<pt_grid, kBlock, 0, ctx->stream>>>(a);
    }
    // 4. second-order network pass and gradient
    MlpTrainArgs t{};
    t.S = m->S;
    t.F = m->F;
    t.L = m->L;
    t.H = m->H;
    t.act = m->act;
    t.T = b->tileT;
    t.QC = b->tileQC;
    t.R = b->tileR;
    t.P = (int)m->per_species_int;
    for (int s = 0; s <= m->S; ++s) {
        t.sp_off[s] = b->groups.off[s];
        t.tile_off[s] = b->tile_off[s];
    }
    t.sp_idx = b->sp_idx;
    t.G = b->G;
    t.w = b->w;
    t.e = b->e;
    t.params = m->params_int;
    t.partial = b->partial;
    const size_t lds = mlp2_lds(t.F, t.H, t.L, t.T, t.QC);
    // gradient in the ABI layout: reduced straight into it, or for a padded
    // model reduced in the padded layout and compacted
    float* gdst = grad ? grad : b->grad;
    if (!grad && m->padded) {
        hipError_t e = hipSuccess;
        gdst = (float*)ctx->ws.get("train.grad_abi", sizeof(float) * (size_t)m->S * m->per_species, &e);
        if (e != hipSuccess) return hip_fail(ctx, e, "gradient workspace");
    }
    float* gred = m->padded ? b->grad : gdst;
    {
        ProfScope ps_(ctx, "train_mlp2");
        // rows per thread and pass: H T / 256 (H and T powers of two), 1 to 4
        const int nr = std::max(1, std::min(4, t.H * t.T / 256));
        using Mlp2 = void (*)(MlpTrainArgs);
        Mlp2 kern = nullptr;
#define TMD_MLP2(TT) \
    if (t.T == TT) kern = nr == 4 ? k_mlp_second<TT, 4> : nr == 2 ? k_mlp_second<TT, 2> : k_mlp_second<TT, 1>;
        TMD_MLP2(8)
        TMD_MLP2(4)
        TMD_MLP2(2)
        TMD_MLP2(1)
#undef TMD_MLP2
        if (!kern) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "no second-order kernel for this tile");
        if (b->tiles > 0) kern<<<(unsigned)b->tiles, 256, lds, ctx->stream>>>(t);
    }
    TMD_HIP(ctx, hipGetLastError());
    {
        GradReduceArgs g{};
        g.S = m->S;
        g.P = (int)m->per_species_int;
        for (int q = 0; q <= m->S; ++q) {
            g.tile_off[q] = b->tile_off[q];
            g.chunk_off[q] = q == 0 ? 0
                                    : g.chunk_off[q - 1] +
                                          (b->tile_off[q] - b->tile_off[q - 1] + kGradChunk - 1) / kGradChunk;
        }
        g.partial = b->partial;
        g.grad = gred;
        ProfScope ps_(ctx, "train_grad_reduce");
        const int pb = (g.P + 255) / 256;
        if (g.chunk_off[m->S] > 0)
            k_grad_chunks<<<(unsigned)(g.chunk_off[m->S] * pb), 256, 0, ctx->stream>>>(g, pb);
        k_grad_reduce<<<blocks_for((int64_t)m->S * m->per_species_int), kBlock, 0, ctx->stream>>>(g);
        if (m->padded)
            k_grad_compact<<<blocks_for((int64_t)m->S * m->per_species), kBlock, 0, ctx->stream>>>(
                m->S, m->per_species, m->per_species_int, param_map(m), gred, gdst);
    }
    TMD_HIP(ctx, hipGetLastError());
    TMD_HIP(ctx, hipMemcpyAsync(ctx->h_totals, b->loss, sizeof(double) * 3, hipMemcpyDeviceToHost, ctx->stream));
    // 5. update
    if (opts->lr > 0.0) {
        const int64_t np = (int64_t)m->S * m->per_species;
        const bool adam = opts->optimizer == TMD_OPT_ADAM;
        if (adam && !m->opt_m) {
            TMD_HIP(ctx, hipMalloc((void**)&m->opt_m, 4 * (size_t)np));
            TMD_HIP(ctx, hipMalloc((void**)&m->opt_v, 4 * (size_t)np));
            TMD_HIP(ctx, hipMemsetAsync(m->opt_m, 0, 4 * (size_t)np, ctx->stream));
            TMD_HIP(ctx, hipMemsetAsync(m->opt_v, 0, 4 * (size_t)np, ctx->stream));
            m->opt_t = 0;
        }
        float c1 = 1.0f, c2 = 1.0f;
        if (adam) {
            m->opt_t += 1;
            c1 = (float)(1.0 - std::pow(opts->beta1, (double)m->opt_t));
            c2 = (float)(1.0 - std::pow(opts->beta2, (double)m->opt_t));
        }
        {
            ProfScope ps_(ctx, "train_update");
            k_optimizer<<<blocks_for(np), kBlock, 0, ctx->stream>>>(np, adam ? 1 : 0, (float)opts->lr,
                                                                     (float)opts->beta1, (float)opts->beta2,
                                                                     (float)opts->eps, c1, c2, gdst, m->params32,
                                                                     m->opt_m, m->opt_v);
        }
        TMD_HIP(ctx, hipGetLastError());
        if ((st = launch_unpack_params(ctx, m)) != TMD_OK) return st;
    }
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < 3; ++q) loss[q] = ctx->h_totals[q];
    return TMD_OK;
}

tmd_status tmd_batch_read(tmd_context* ctx, const tmd_batch* b, int32_t field, float* out) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (!b || !out) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null argument");
    const float* src = nullptr;
    size_t n = 0;
    bool rows = false;  // [N][F] rows: the model's own features
    switch (field) {
        case TMD_BATCH_G: src = b->G, rows = true; break;
        case TMD_BATCH_ENERGY: src = b->Ei, n = (size_t)b->N; break;
        case TMD_BATCH_FORCES: src = b->Fp, n = (size_t)b->N * 3; break;
        case TMD_BATCH_RESIDUAL: src = b->r, n = (size_t)b->N * 3; break;
        case TMD_BATCH_TANGENT: src = b->w, rows = true; break;
        default: return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "unknown batch field");
    }
    if (rows) {
        tmd_status st = launch_compact_features(ctx, b->N, src, b->F, b->Fabi, b->K, b->Kabi, b->M + 1, out);
        if (st != TMD_OK) return st;
    } else {
        TMD_HIP(ctx, hipMemcpyAsync(out, src, 4 * n, hipMemcpyDeviceToDevice, ctx->stream));
    }
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return TMD_OK;
}

}  // extern "C"

namespace tmd {

tmd_status launch_unpack_params(tmd_context* ctx, tmd_model* m) {
    UnpackArgs u{};
    u.S = m->S;
    u.L = m->L;
    u.H = m->H;
    u.Fpad = m->Fpad;
    u.P = m->per_species;
    u.P_int = m->per_species_int;
    u.wstride = m->w_species_stride;
    for (int l = 0; l < m->L; ++l) {
        u.w_off[l] = m->w_off[l];
        u.wt_off[l] = m->wt_off[l];
    }
    u.pm = param_map(m);
    u.params = m->params32;
    u.params_int = m->padded ? m->params_int : nullptr;
    u.w32 = m->w32;
    u.wbf = m->wbf;
    u.bias = m->bias;
    u.wout = m->wout;
    u.bout = m->bout;
    k_unpack<<<blocks_for((int64_t)m->S * m->per_species), kBlock, 0, ctx->stream>>>(u);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd
