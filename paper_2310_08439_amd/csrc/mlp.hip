// Per-element MLP: atomic energies E_a = NNP_s(G_a) and their input gradient
// dE_a/dG_a by back-propagation (Sec. III.A; the paper fuses forward and
// backward of the dense network into one kernel and keeps both W and W^T,
// which is also done here: the backward GEMMs read stored transposes so that
// every MFMA operand load is contiguous).
//
// All GEMMs run on MFMA in the transposed orientation Z^T = W A^T: hidden
// units are the MFMA rows and 16 atoms form the MFMA columns.  With that
// orientation the accumulator layout of one layer (lane = (row group, atom),
// four consecutive rows per lane) is exactly the B-operand layout the next
// layer needs, up to a fixed permutation of the reduction index that is
// applied identically to the weights.  Activations therefore never leave
// registers between layers.
//   BF16: v_mfma_f32_16x16x32_bf16, operands rounded to BF16 (nearest-even),
//         FP32 accumulation.  One K-step covers 32 hidden units: for lane
//         group g the 8 operand slots hold units {4g..4g+3, 16+4g..16+4g+3}.
//   FP32: v_mfma_f32_16x16x4_f32.  One K-step covers 4 units, lane group g
//         holding unit 16*blk + 4g + r in step (blk, r).
// Atoms of one species are processed together through the species index
// list built with the neighbour list.
#include "tmd_internal.h"

namespace tmd {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

struct MlpArgs {
    int S, F, Fpad, act;
    int64_t sp_off[kMaxSpecies + 1];
    int64_t tile_off[kMaxSpecies + 1];
    const int32_t* sp_idx;
    const float* G;
    float* Ei;
    float* dG;
    const float* w32;
    const __hip_bfloat16* wbf;
    int64_t wstride;
    int64_t w_off[TMD_MAX_HIDDEN];
    int64_t wt_off[TMD_MAX_HIDDEN];
    const float* bias;  // [S][L][H]
    const float* wout;  // [S][H]
    const float* bout;  // [S]
    int L;
};

__device__ __forceinline__ float act_f(int act, float z) {
    if (act == TMD_ACT_SQUAREPLUS) return 0.5f * (z + __builtin_sqrtf(z * z + 4.0f));
    // tanh(z) = 1 - 2/(exp(2z)+1); saturates cleanly to +-1
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * z);
    return 1.0f - 2.0f / (e + 1.0f);
}
__device__ __forceinline__ float act_df(int act, float z, float a) {
    if (act == TMD_ACT_SQUAREPLUS) return 0.5f * (1.0f + z * __builtin_amdgcn_rsqf(z * z + 4.0f));
    return 1.0f - a * a;
}

__device__ __forceinline__ bf16x4 load_bf4(const __hip_bfloat16* p) {
    return *reinterpret_cast<const bf16x4*>(p);
}
__device__ __forceinline__ bf16x8 cat8(bf16x4 lo, bf16x4 hi) {
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}
__device__ __forceinline__ bf16x4 to_bf4(f32x4 v) {
    bf16x4 r;
    r[0] = (__bf16)v[0];
    r[1] = (__bf16)v[1];
    r[2] = (__bf16)v[2];
    r[3] = (__bf16)v[3];
    return r;
}

// One wave: CB column blocks of 16 atoms of species s.
template <bool BF16, int H, int L, int CB>
__global__ void __launch_bounds__(256) k_mlp(MlpArgs a) {
    constexpr int NB = H / 16;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int s = -1;
    for (int q = 0; q < a.S; ++q)
        if (wave >= a.tile_off[q] && wave < a.tile_off[q + 1]) s = q;
    if (s < 0) return;
    const int64_t first = a.sp_off[s] + (wave - a.tile_off[s]) * (16 * CB);
    const int64_t end = a.sp_off[s + 1];
    int64_t atom[CB];
    bool valid[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int64_t r = first + cb * 16 + col;
        valid[cb] = r < end;
        atom[cb] = valid[cb] ? (int64_t)a.sp_idx[r] : 0;
    }
    const float* w32 = a.w32 + s * a.wstride;
    const __hip_bfloat16* wbf = a.wbf + s * a.wstride;
    const float* bias = a.bias + (int64_t)s * L * H;

    f32x4 acc[NB][CB];
    f32x4 dact[L][NB][CB];

    // ---- layer 1: Z1^T = W1 G^T + b1
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
        const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + 16 * ob + 4 * grp);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = bv;
    }
    if constexpr (BF16) {
        for (int k0 = 0; k0 < a.Fpad; k0 += 32) {
            bf16x8 bop[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                f32x4 lo = {0, 0, 0, 0}, hi = {0, 0, 0, 0};
                const int c0 = k0 + 4 * grp, c1 = k0 + 16 + 4 * grp;
                if (valid[cb] && c0 < a.F) lo = *reinterpret_cast<const f32x4*>(a.G + atom[cb] * a.F + c0);
                if (valid[cb] && c1 < a.F) hi = *reinterpret_cast<const f32x4*>(a.G + atom[cb] * a.F + c1);
                bop[cb] = cat8(to_bf4(lo), to_bf4(hi));
            }
#pragma unroll
            for (int ob = 0; ob < NB; ++ob) {
                const __hip_bfloat16* wr = wbf + a.w_off[0] + (int64_t)(16 * ob + col) * a.Fpad + k0 + 4 * grp;
                const bf16x8 av = cat8(load_bf4(wr), load_bf4(wr + 16));
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc[ob][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[cb], acc[ob][cb], 0, 0, 0);
            }
        }
    } else {
        for (int k0 = 0; k0 < a.Fpad; k0 += 16) {
            f32x4 bv[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                bv[cb] = f32x4{0, 0, 0, 0};
                const int c0 = k0 + 4 * grp;
                if (valid[cb] && c0 < a.F) bv[cb] = *reinterpret_cast<const f32x4*>(a.G + atom[cb] * a.F + c0);
            }
#pragma unroll
            for (int ob = 0; ob < NB; ++ob) {
                const f32x4 wv =
                    *reinterpret_cast<const f32x4*>(w32 + a.w_off[0] + (int64_t)(16 * ob + col) * a.Fpad + k0 + 4 * grp);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[ob][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[r], bv[cb][r], acc[ob][cb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[ob][cb][r];
                const float y = act_f(a.act, z);
                dact[0][ob][cb][r] = act_df(a.act, z, y);
                acc[ob][cb][r] = y;
            }

    // ---- hidden layers 2..L: Z_l^T = W_l A_{l-1}^T + b_l
    auto layer = [&](const float* w32l, const __hip_bfloat16* wbfl, const float* bl, bool add_bias) {
        // snapshot the previous activations as B operands
        if constexpr (BF16) {
            bf16x8 bop[NB / 2][CB];
#pragma unroll
            for (int s2 = 0; s2 < NB / 2; ++s2)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) bop[s2][cb] = cat8(to_bf4(acc[2 * s2][cb]), to_bf4(acc[2 * s2 + 1][cb]));
#pragma unroll
            for (int ob = 0; ob < NB; ++ob) {
                f32x4 init = {0, 0, 0, 0};
                if (add_bias) init = *reinterpret_cast<const f32x4*>(bl + 16 * ob + 4 * grp);
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = init;
            }
#pragma unroll
            for (int s2 = 0; s2 < NB / 2; ++s2)
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) {
                    const __hip_bfloat16* wr = wbfl + (int64_t)(16 * ob + col) * H + 32 * s2 + 4 * grp;
                    const bf16x8 av = cat8(load_bf4(wr), load_bf4(wr + 16));
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[ob][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[s2][cb], acc[ob][cb], 0, 0, 0);
                }
        } else {
            f32x4 xin[NB][CB];
#pragma unroll
            for (int ob = 0; ob < NB; ++ob)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) xin[ob][cb] = acc[ob][cb];
#pragma unroll
            for (int ob = 0; ob < NB; ++ob) {
                f32x4 init = {0, 0, 0, 0};
                if (add_bias) init = *reinterpret_cast<const f32x4*>(bl + 16 * ob + 4 * grp);
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = init;
            }
#pragma unroll
            for (int blk = 0; blk < NB; ++blk)
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) {
                    const f32x4 wv =
                        *reinterpret_cast<const f32x4*>(w32l + (int64_t)(16 * ob + col) * H + 16 * blk + 4 * grp);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            acc[ob][cb] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(wv[r], xin[blk][cb][r], acc[ob][cb], 0, 0, 0);
                }
        }
    };

#pragma unroll
    for (int l = 1; l < L; ++l) {
        layer(w32 + a.w_off[l], wbf + a.w_off[l], bias + l * H, true);
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[ob][cb][r];
                    const float y = act_f(a.act, z);
                    dact[l][ob][cb][r] = act_df(a.act, z, y);
                    acc[ob][cb][r] = y;
                }
    }

    // ---- output layer: E = w_out . a_L + b_out; delta_L = w_out * act'(z_L)
    const float* wo = a.wout + (int64_t)s * H;
    float e[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) e[cb] = 0.0f;
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
        const f32x4 wv = *reinterpret_cast<const f32x4*>(wo + 16 * ob + 4 * grp);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                e[cb] = fmaf(wv[r], acc[ob][cb][r], e[cb]);
                acc[ob][cb][r] = wv[r] * dact[L - 1][ob][cb][r];
            }
    }
    const float bo = a.bout[s];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        float v = e[cb];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (grp == 0 && valid[cb]) a.Ei[atom[cb]] = v + bo;
    }

    // ---- backward through hidden layers: delta_{l-1} = (W_l^T delta_l) * act'(z_{l-1})
#pragma unroll
    for (int l = L - 1; l >= 1; --l) {
        layer(w32 + a.wt_off[l], wbf + a.wt_off[l], nullptr, false);
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[ob][cb][r] *= dact[l - 1][ob][cb][r];
    }

    // ---- dE/dG^T = W_1^T delta_1 : F output rows in blocks of 16
    if constexpr (BF16) {
        bf16x8 bop[NB / 2][CB];
#pragma unroll
        for (int s2 = 0; s2 < NB / 2; ++s2)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) bop[s2][cb] = cat8(to_bf4(acc[2 * s2][cb]), to_bf4(acc[2 * s2 + 1][cb]));
        for (int fb = 0; fb < a.Fpad / 16; ++fb) {
            f32x4 out[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) out[cb] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int s2 = 0; s2 < NB / 2; ++s2) {
                const __hip_bfloat16* wr = wbf + a.wt_off[0] + (int64_t)(16 * fb + col) * H + 32 * s2 + 4 * grp;
                const bf16x8 av = cat8(load_bf4(wr), load_bf4(wr + 16));
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    out[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[s2][cb], out[cb], 0, 0, 0);
            }
            const int f0 = 16 * fb + 4 * grp;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                if (valid[cb] && f0 < a.F) *reinterpret_cast<f32x4*>(a.dG + atom[cb] * a.F + f0) = out[cb];
        }
    } else {
        for (int fb = 0; fb < a.Fpad / 16; ++fb) {
            f32x4 out[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) out[cb] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
                const f32x4 wv =
                    *reinterpret_cast<const f32x4*>(w32 + a.wt_off[0] + (int64_t)(16 * fb + col) * H + 16 * blk + 4 * grp);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        out[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[r], acc[blk][cb][r], out[cb], 0, 0, 0);
            }
            const int f0 = 16 * fb + 4 * grp;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                if (valid[cb] && f0 < a.F) *reinterpret_cast<f32x4*>(a.dG + atom[cb] * a.F + f0) = out[cb];
        }
    }
}

using MlpFn = void (*)(MlpArgs);

template <bool BF16, int H>
MlpFn pick_L(int L, int* cb) {
    switch (L) {
        case 1: *cb = 2; return k_mlp<BF16, H, 1, 2>;
        case 2: *cb = 2; return k_mlp<BF16, H, 2, 2>;
        case 3: *cb = 1; return k_mlp<BF16, H, 3, 1>;
        default: *cb = 1; return k_mlp<BF16, H, 4, 1>;
    }
}

template <bool BF16>
MlpFn pick_H(int H, int L, int* cb) {
    switch (H) {
        case 32: return pick_L<BF16, 32>(L, cb);
        case 64: return pick_L<BF16, 64>(L, cb);
        default: return pick_L<BF16, 128>(L, cb);
    }
}

}  // namespace

tmd_status launch_mlp(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, const float* G, float* Ei,
                      float* dG) {
    MlpArgs a{};
    a.S = m->S;
    a.F = m->F;
    a.Fpad = m->Fpad;
    a.act = m->act;
    a.L = m->L;
    int cb = 1;
    MlpFn fn = (m->prec == TMD_BF16_MLP) ? pick_H<true>(m->H, m->L, &cb) : pick_H<false>(m->H, m->L, &cb);
    const int apw = 16 * cb;
    int64_t tiles = 0;
    for (int s = 0; s < m->S; ++s) {
        a.sp_off[s] = nl->sp_off[s];
        a.tile_off[s] = tiles;
        tiles += (nl->sp_count[s] + apw - 1) / apw;
    }
    a.sp_off[m->S] = nl->sp_off[m->S];
    a.tile_off[m->S] = tiles;
    a.sp_idx = nl->sp_idx;
    a.G = G;
    a.Ei = Ei;
    a.dG = dG;
    a.w32 = m->w32;
    a.wbf = m->wbf;
    a.wstride = m->w_species_stride;
    for (int l = 0; l < m->L; ++l) {
        a.w_off[l] = m->w_off[l];
        a.wt_off[l] = m->wt_off[l];
    }
    a.bias = m->bias;
    a.wout = m->wout;
    a.bout = m->bout;
    if (tiles == 0) return TMD_OK;
    const unsigned grid = (unsigned)((tiles + 3) / 4);
    {
        ProfScope ps_(ctx, "mlp");
        fn<<<grid, 256, 0, ctx->stream>>>(a);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd
