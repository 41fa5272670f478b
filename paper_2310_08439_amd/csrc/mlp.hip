// Per-element MLP: atomic energies E_a = NNP_s(G_a) and their input gradient
// dE_a/dG_a by back-propagation (Sec. III.A; the paper fuses forward and
// backward of the dense network into one kernel and keeps both W and W^T,
// which is also done here: the backward GEMMs read stored transposes so that
// every operand row is contiguous).
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
// A workgroup of 4 or 8 waves takes 128 atoms of one species; each
// layer's weights (forward or transposed) are staged once per workgroup into
// LDS in column chunks with padded rows, and all four waves read their MFMA
// A operands from there.
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
    const float* G;      // FP32 descriptors (FP32 kernels)
    const uint16_t* Gb;  // BF16 descriptors, the bits of (__bf16)G (BF16 kernels)
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

template <bool BF16>
struct WT;
template <>
struct WT<true> {
    using T = __hip_bfloat16;
    // elements of row padding in LDS: rows 2 (mod 32) words apart, so that the
    // 16 rows an A-operand read touches (8 bytes per lane) fall on distinct
    // banks (with 8 elements, 4 words mod 32, every read was a two-way
    // conflict: 7.8 conflict cycles per LDS instruction in the resident
    // kernel, 0.06 with 4)
    static constexpr int kPad = 4;
    static constexpr int kChunk = 128;  // columns staged at a time
};
template <>
struct WT<false> {
    using T = float;
    // measured at 1 M atoms (96-128-128-1, FP32): 1.31 ms with 4 elements of
    // row padding (and with 44, 52 or 60), 1.03 ms with 20, 24, 28 or 36 (the
    // staged tile is then 43-51 KB: three workgroups per CU instead of four)
    static constexpr int kPad = 28;
    static constexpr int kChunk = 64;
};

// LDS capacity in elements: 128 rows x (chunk + pad).
template <bool BF16>
constexpr int lds_elems() {
    return 128 * (WT<BF16>::kChunk + WT<BF16>::kPad);
}

template <int ACT>
__device__ __forceinline__ float act_f(float z) {
    constexpr int act = ACT;
    if constexpr (act == TMD_ACT_SQUAREPLUS) return 0.5f * (z + __builtin_amdgcn_sqrtf(z * z + 4.0f));
    // tanh(z) = 1 - 2/(exp(2z)+1) with the hardware reciprocal (1 ulp); saturates
    // cleanly to +-1 (exp2 overflows to inf, whose reciprocal is 0)
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * z);
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}
template <int ACT>
__device__ __forceinline__ float act_df(float z, float a) {
    constexpr int act = ACT;
    if constexpr (act == TMD_ACT_SQUAREPLUS) return 0.5f * (1.0f + z * __builtin_amdgcn_rsqf(z * z + 4.0f));
    return 1.0f - a * a;
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

// Stage rows [0, nrows) x columns [c0, c0 + nc) of a row-major matrix with
// `ld` elements per row into LDS rows of stride nc + pad.  All threads of the
// workgroup take part; callers synchronise around it.
template <bool BF16>
__device__ __forceinline__ void stage(const typename WT<BF16>::T* W, int ld, int nrows, int c0, int nc,
                                      typename WT<BF16>::T* lds) {
    using T = typename WT<BF16>::T;
    constexpr int V = 16 / sizeof(T);
    const int per_row = nc / V, stride = nc + WT<BF16>::kPad;
    for (int c = threadIdx.x; c < nrows * per_row; c += blockDim.x) {
        const int r = c / per_row, k = (c - r * per_row) * V;
        // rows are 8-byte aligned in LDS (not 16: see kPad)
        const uint4 v = *reinterpret_cast<const uint4*>(W + (int64_t)r * ld + c0 + k);
        uint2* d = reinterpret_cast<uint2*>(lds + r * stride + k);
        d[0] = make_uint2(v.x, v.y);
        d[1] = make_uint2(v.z, v.w);
    }
}

// B operand of the first layer: four consecutive features of one atom's
// descriptor row, zero past the row's end.
__device__ __forceinline__ f32x4 load_g4(const float* G, int64_t atom, int F, int g0, bool valid) {
    f32x4 v = {0, 0, 0, 0};
    if (!valid || g0 >= F) return v;
    const float* row = G + atom * F;
    if ((F & 3) == 0) return *reinterpret_cast<const f32x4*>(row + g0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (g0 + r < F) v[r] = row[g0 + r];
    return v;
}

// The same four features stored as BF16 (rounded by the producer exactly as
// to_bf4 rounds: nearest-even), so the operand bits are those of
// to_bf4(load_g4(...)) on the FP32 row.
__device__ __forceinline__ bf16x4 load_gb4(const uint16_t* Gb, int64_t atom, int F, int g0, bool valid) {
    if (!valid || g0 >= F) return bf16x4{0, 0, 0, 0};
    const uint16_t* row = Gb + atom * F;
    if ((F & 3) == 0) return __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2*>(row + g0));
    bf16x4 v = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (g0 + r < F) v[r] = __builtin_bit_cast(__bf16, row[g0 + r]);
    return v;
}

__device__ __forceinline__ void store_dg4(float* dG, int64_t atom, int F, int f0, bool valid, f32x4 v) {
    if (!valid || f0 >= F) return;
    float* row = dG + atom * F;
    if ((F & 3) == 0) {
        *reinterpret_cast<f32x4*>(row + f0) = v;
        return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (f0 + r < F) row[f0 + r] = v[r];
}

// Hidden layer (H x H): acc[ob][cb] += W x, x held in the accumulator layout
// of the previous layer.  W is row-major [H][H] in global memory, staged
// through LDS in CH-column chunks; all indices are compile-time.
template <bool BF16, int H, int CB>
__device__ __forceinline__ void dense_hidden(const typename WT<BF16>::T* W, typename WT<BF16>::T* lds,
                                             const f32x4 (&x)[H / 16][CB], f32x4 (&acc)[H / 16][CB]) {
    using T = typename WT<BF16>::T;
    constexpr int NB = H / 16;
    constexpr int CH = WT<BF16>::kChunk < H ? WT<BF16>::kChunk : H;
    constexpr int stride = CH + WT<BF16>::kPad;
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int c0 = 0; c0 < H; c0 += CH) {
        __syncthreads();
        stage<BF16>(W, H, H, c0, CH, lds);
        __syncthreads();
        if constexpr (BF16) {
#pragma unroll
            for (int k0 = 0; k0 < CH; k0 += 32) {
                const int blk = (c0 + k0) / 16;
                bf16x8 bop[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) bop[cb] = cat8(to_bf4(x[blk][cb]), to_bf4(x[blk + 1][cb]));
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) {
                    const T* wr = lds + (16 * ob + col) * stride + k0 + 4 * grp;
                    const bf16x8 av =
                        cat8(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16));
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[ob][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[cb], acc[ob][cb], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int k0 = 0; k0 < CH; k0 += 16) {
                const int blk = (c0 + k0) / 16;
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) {
                    const f32x4 wv = *reinterpret_cast<const f32x4*>(lds + (16 * ob + col) * stride + k0 + 4 * grp);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            acc[ob][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[r], x[blk][cb][r], acc[ob][cb], 0, 0, 0);
                }
            }
        }
    }
}

template <bool BF16, int H, int L, int CB, int ACT, int NW>
__global__ void __launch_bounds__(64 * NW) k_mlp(MlpArgs a) {
    constexpr int NB = H / 16;
    constexpr int kTile = NW * 16 * CB;
    using T = typename WT<BF16>::T;
    constexpr int PAD = WT<BF16>::kPad, CHUNK = WT<BF16>::kChunk;
    __shared__ __attribute__((aligned(16))) T lds[lds_elems<BF16>()];
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t tile = blockIdx.x;
    int s = 0;
    for (int q = 0; q < a.S; ++q)
        if (tile >= a.tile_off[q] && tile < a.tile_off[q + 1]) s = q;
    const int64_t first = a.sp_off[s] + (tile - a.tile_off[s]) * kTile + (threadIdx.x >> 6) * (16 * CB);
    const int64_t end = a.sp_off[s + 1];
    int64_t atom[CB];
    bool valid[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int64_t r = first + cb * 16 + col;
        valid[cb] = r < end;
        atom[cb] = valid[cb] ? (int64_t)a.sp_idx[r] : 0;
    }
    const T* wsp;
    if constexpr (BF16) wsp = a.wbf + s * a.wstride;
    else wsp = a.w32 + s * a.wstride;
    const float* bias = a.bias + (int64_t)s * L * H;

    f32x4 acc[NB][CB];
    f32x4 x[NB][CB];
    f32x4 dact[L][NB][CB];

    auto set_bias = [&](const float* bl) {
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) {
            f32x4 init = {0, 0, 0, 0};
            if (bl) init = *reinterpret_cast<const f32x4*>(bl + 16 * ob + 4 * grp);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = init;
        }
    };
    auto activate = [&](int l) {
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[ob][cb][r];
                    const float y = act_f<ACT>(z);
                    dact[l][ob][cb][r] = act_df<ACT>(z, y);
                    acc[ob][cb][r] = y;
                }
    };
    auto keep = [&]() {
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) x[ob][cb] = acc[ob][cb];
    };

    // ---- layer 1: W_1 [H][Fpad] times G^T, weights staged in column chunks
    set_bias(bias);
    {
        const T* W = wsp + a.w_off[0];
        for (int c0 = 0; c0 < a.Fpad; c0 += CHUNK) {
            const int nc = min(CHUNK, a.Fpad - c0);
            const int stride = nc + PAD;
            __syncthreads();
            stage<BF16>(W, a.Fpad, H, c0, nc, lds);
            __syncthreads();
            if constexpr (BF16) {
                for (int k0 = 0; k0 < nc; k0 += 32) {
                    bf16x8 bop[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const int g0 = c0 + k0 + 4 * grp;
                        bop[cb] = cat8(load_gb4(a.Gb, atom[cb], a.F, g0, valid[cb]),
                                       load_gb4(a.Gb, atom[cb], a.F, g0 + 16, valid[cb]));
                    }
#pragma unroll
                    for (int ob = 0; ob < NB; ++ob) {
                        const T* wr = lds + (16 * ob + col) * stride + k0 + 4 * grp;
                        const bf16x8 av =
                            cat8(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16));
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            acc[ob][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[cb], acc[ob][cb], 0, 0, 0);
                    }
                }
            } else {
                for (int k0 = 0; k0 < nc; k0 += 16) {
                    f32x4 bv[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) bv[cb] = load_g4(a.G, atom[cb], a.F, c0 + k0 + 4 * grp, valid[cb]);
#pragma unroll
                    for (int ob = 0; ob < NB; ++ob) {
                        const f32x4 wv =
                            *reinterpret_cast<const f32x4*>(lds + (16 * ob + col) * stride + k0 + 4 * grp);
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[ob][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[r], bv[cb][r], acc[ob][cb], 0, 0, 0);
                    }
                }
            }
        }
    }
    activate(0);
    // ---- hidden layers 2..L
#pragma unroll
    for (int l = 1; l < L; ++l) {
        keep();
        set_bias(bias + l * H);
        dense_hidden<BF16, H, CB>(wsp + a.w_off[l], lds, x, acc);
        activate(l);
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
        keep();
        set_bias(nullptr);
        dense_hidden<BF16, H, CB>(wsp + a.wt_off[l], lds, x, acc);
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[ob][cb][r] *= dact[l - 1][ob][cb][r];
    }

    // ---- dE/dG^T = W_1^T delta_1: Fpad output rows; W_1^T [Fpad][H] is
    // staged in panels of PR full rows.
    constexpr int NS = NB / 2 > 0 ? NB / 2 : 1;
    bf16x8 bop[NS][CB];
    if constexpr (BF16) {
#pragma unroll
        for (int s2 = 0; s2 < NB / 2; ++s2)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) bop[s2][cb] = cat8(to_bf4(acc[2 * s2][cb]), to_bf4(acc[2 * s2 + 1][cb]));
    }
    const T* w1t = wsp + a.wt_off[0];
    constexpr int PR = lds_elems<BF16>() / (H + PAD) / 16 * 16;
    for (int r0 = 0; r0 < a.Fpad; r0 += PR) {
        const int nr = min(PR, a.Fpad - r0);
        __syncthreads();
        stage<BF16>(w1t + (int64_t)r0 * H, H, nr, 0, H, lds);
        __syncthreads();
        for (int fb = 0; fb < nr / 16; ++fb) {
            f32x4 out[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) out[cb] = f32x4{0, 0, 0, 0};
            if constexpr (BF16) {
#pragma unroll
                for (int s2 = 0; s2 < NB / 2; ++s2) {
                    const T* wr = lds + (16 * fb + col) * (H + PAD) + 32 * s2 + 4 * grp;
                    const bf16x8 av =
                        cat8(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16));
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        out[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[s2][cb], out[cb], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int blk = 0; blk < NB; ++blk) {
                    const f32x4 wv =
                        *reinterpret_cast<const f32x4*>(lds + (16 * fb + col) * (H + PAD) + 16 * blk + 4 * grp);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            out[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[r], acc[blk][cb][r], out[cb], 0, 0, 0);
                }
            }
            const int f0 = r0 + 16 * fb + 4 * grp;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) store_dg4(a.dG, atom[cb], a.F, f0, valid[cb], out[cb]);
        }
    }
}

// Resident-weight form (BF16, networks whose weights fit in LDS): one
// workgroup of 16 waves per CU keeps every matrix of one species in LDS
// (W_1, the hidden W_l, their transposes and W_1^T, padded rows) and its waves
// take 16-atom tiles independently, with no barrier between layers.  The
// weights are staged once per species and workgroup instead of once per
// 128-atom tile (at 1 M atoms that is ~30 MB of L2 traffic instead of ~0.9 GB).
template <int H, int L>
constexpr int resident_rows_elems(int Fpad) {
    return H * (Fpad + WT<true>::kPad) + 2 * (L - 1) * H * (H + WT<true>::kPad) + Fpad * (H + WT<true>::kPad);
}

template <int H, int L, int ACT>
__global__ void __launch_bounds__(1024) k_mlp_resident(MlpArgs a) {
    using T = __hip_bfloat16;
    constexpr int NB = H / 16, PAD = WT<true>::kPad;
    extern __shared__ __attribute__((aligned(16))) T sw[];
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4, wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int s1 = a.Fpad + PAD, sh = H + PAD;
    T* W1 = sw;                        // [H][Fpad + PAD]
    T* Wh = W1 + H * s1;               // L-1 x [H][H + PAD]
    T* Wt = Wh + (L - 1) * H * sh;     // L-1 x [H][H + PAD], transposed hidden layers
    T* W1t = Wt + (L - 1) * H * sh;    // [Fpad][H + PAD]
    for (int s = 0; s < a.S; ++s) {
        const int64_t first_atom = a.sp_off[s], end = a.sp_off[s + 1];
        const int64_t ntiles = (end - first_atom + 15) / 16;
        if (ntiles == 0) continue;  // uniform over the workgroup
        const T* wsp = a.wbf + s * a.wstride;
        __syncthreads();  // the previous species' tiles are done with the LDS copy
        stage<true>(wsp + a.w_off[0], a.Fpad, H, 0, a.Fpad, W1);
        for (int l = 1; l < L; ++l) {
            stage<true>(wsp + a.w_off[l], H, H, 0, H, Wh + (l - 1) * H * sh);
            stage<true>(wsp + a.wt_off[l], H, H, 0, H, Wt + (l - 1) * H * sh);
        }
        stage<true>(wsp + a.wt_off[0], H, a.Fpad, 0, H, W1t);
        __syncthreads();
        const float* bias = a.bias + (int64_t)s * L * H;
        const float* wo = a.wout + (int64_t)s * H;
        const float bo = a.bout[s];
        for (int64_t tile = (int64_t)blockIdx.x * nw + wv; tile < ntiles; tile += (int64_t)gridDim.x * nw) {
            // keep the weight reads inside the tile loop (hoisting them out of
            // it would pin every weight fragment in registers)
            __asm__ volatile("" ::: "memory");
            const int64_t r = first_atom + tile * 16 + col;
            const bool valid = r < end;
            const int64_t atom = valid ? (int64_t)a.sp_idx[r] : 0;
            f32x4 acc[NB], x[NB], dact[L][NB];
            auto set_bias = [&](const float* bl) {
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) {
                    f32x4 init = {0, 0, 0, 0};
                    if (bl) init = *reinterpret_cast<const f32x4*>(bl + 16 * ob + 4 * grp);
                    acc[ob] = init;
                }
            };
            auto activate = [&](int l) {
#pragma unroll
                for (int ob = 0; ob < NB; ++ob)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float z = acc[ob][q];
                        const float y = act_f<ACT>(z);
                        dact[l][ob][q] = act_df<ACT>(z, y);
                        acc[ob][q] = y;
                    }
            };
            // A operand rows of a resident matrix times the B operand held in x
            auto dense = [&](const T* Wm) {
#pragma unroll
                for (int k0 = 0; k0 < H; k0 += 32) {
                    const int blk = k0 / 16;
                    const bf16x8 bop = cat8(to_bf4(x[blk]), to_bf4(x[blk + 1]));
#pragma unroll
                    for (int ob = 0; ob < NB; ++ob) {
                        const T* wr = Wm + (16 * ob + col) * sh + k0 + 4 * grp;
                        const bf16x8 av =
                            cat8(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16));
                        acc[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop, acc[ob], 0, 0, 0);
                    }
                }
            };
            // layer 1
            set_bias(bias);
            for (int k0 = 0; k0 < a.Fpad; k0 += 32) {
                const int g0 = k0 + 4 * grp;
                const bf16x8 bop = cat8(load_gb4(a.Gb, atom, a.F, g0, valid), load_gb4(a.Gb, atom, a.F, g0 + 16, valid));
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) {
                    const T* wr = W1 + (16 * ob + col) * s1 + k0 + 4 * grp;
                    const bf16x8 av =
                        cat8(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16));
                    acc[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop, acc[ob], 0, 0, 0);
                }
            }
            activate(0);
#pragma unroll
            for (int l = 1; l < L; ++l) {
                __asm__ volatile("" ::: "memory");  // one layer's weights in flight at a time
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) x[ob] = acc[ob];
                set_bias(bias + l * H);
                dense(Wh + (l - 1) * H * sh);
                activate(l);
            }
            // output layer and its adjoint
            float e = 0.0f;
#pragma unroll
            for (int ob = 0; ob < NB; ++ob) {
                const f32x4 wvv = *reinterpret_cast<const f32x4*>(wo + 16 * ob + 4 * grp);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    e = fmaf(wvv[q], acc[ob][q], e);
                    acc[ob][q] = wvv[q] * dact[L - 1][ob][q];
                }
            }
            e += __shfl_xor(e, 16);
            e += __shfl_xor(e, 32);
            if (grp == 0 && valid) a.Ei[atom] = e + bo;
            // backward through the hidden layers
#pragma unroll
            for (int l = L - 1; l >= 1; --l) {
                __asm__ volatile("" ::: "memory");
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) x[ob] = acc[ob];
                set_bias(nullptr);
                dense(Wt + (l - 1) * H * sh);
#pragma unroll
                for (int ob = 0; ob < NB; ++ob)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[ob][q] *= dact[l - 1][ob][q];
            }
            // dE/dG^T = W_1^T delta_1
            __asm__ volatile("" ::: "memory");
            bf16x8 bop[NB / 2];
#pragma unroll
            for (int s2 = 0; s2 < NB / 2; ++s2) bop[s2] = cat8(to_bf4(acc[2 * s2]), to_bf4(acc[2 * s2 + 1]));
            for (int fb = 0; fb < a.Fpad / 16; ++fb) {
                f32x4 out = {0, 0, 0, 0};
#pragma unroll
                for (int s2 = 0; s2 < NB / 2; ++s2) {
                    const T* wr = W1t + (16 * fb + col) * sh + 32 * s2 + 4 * grp;
                    const bf16x8 av =
                        cat8(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16));
                    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[s2], out, 0, 0, 0);
                }
                store_dg4(a.dG, atom, a.F, 16 * fb + 4 * grp, valid, out);
            }
        }
    }
}

using ResidentFn = void (*)(MlpArgs);
template <int ACT>
ResidentFn pick_resident(int H, int L) {
    if (H == 128 && L == 1) return k_mlp_resident<128, 1, ACT>;
    if (H == 128 && L == 2) return k_mlp_resident<128, 2, ACT>;
    if (H == 64 && L == 2) return k_mlp_resident<64, 2, ACT>;
    if (H == 64 && L == 3) return k_mlp_resident<64, 3, ACT>;
    return nullptr;
}
int resident_lds_bytes(int H, int L, int Fpad) {
    const int pad = 4;
    return 2 * (H * (Fpad + pad) + 2 * (L - 1) * H * (H + pad) + Fpad * (H + pad));
}
constexpr int kMaxResidentLds = 150 * 1024;

using MlpFn = void (*)(MlpArgs);

// Shape of a workgroup: W waves of CB 16-atom column blocks each.  H <= 64:
// 4 waves x 2 blocks.  H = 128: 1 block per wave, so that a wave's
// activations and derivatives fit in far fewer registers (4 waves per SIMD
// for two hidden layers), with 8 waves per workgroup so that each staged
// weight panel is still shared by 128 atoms.
struct MlpShape {
    MlpFn fn;
    int cb, waves;
};

template <bool BF16, int H, int ACT>
MlpShape pick_L(int L) {
    constexpr int C = (H == 128) ? 1 : 2;
    constexpr int W = (H == 128) ? 8 : 4;  // deeper H = 128 nets: 4 waves, up to 512 registers
    switch (L) {
        case 1: return {k_mlp<BF16, H, 1, C, ACT, W>, C, W};
        case 2: return {k_mlp<BF16, H, 2, C, ACT, W>, C, W};
        case 3: return {k_mlp<BF16, H, 3, C, ACT, 4>, C, 4};
        default: return {k_mlp<BF16, H, 4, C, ACT, 4>, C, 4};
    }
}

template <bool BF16, int ACT>
MlpShape pick_H(int H, int L) {
    switch (H) {
        case 32: return pick_L<BF16, 32, ACT>(L);
        case 64: return pick_L<BF16, 64, ACT>(L);
        default: return pick_L<BF16, 128, ACT>(L);
    }
}

template <bool BF16>
MlpShape pick_act(int act, int H, int L) {
    return act == TMD_ACT_SQUAREPLUS ? pick_H<BF16, TMD_ACT_SQUAREPLUS>(H, L) : pick_H<BF16, TMD_ACT_TANH>(H, L);
}

}  // namespace

SpeciesGroups species_groups(const tmd_nlist* nl) {
    SpeciesGroups g;
    g.S = nl->S;
    for (int s = 0; s <= nl->S; ++s) g.off[s] = nl->sp_off[s];
    g.idx = nl->sp_idx;
    return g;
}

tmd_status launch_mlp(tmd_context* ctx, const tmd_model* m, const SpeciesGroups& g, tmd_precision prec,
                      const float* G, const uint16_t* Gb, float* Ei, float* dG) {
    if ((prec == TMD_BF16_MLP) != (Gb != nullptr))
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "BF16 MLP without BF16 descriptors, or the reverse");
    MlpArgs a{};
    a.S = m->S;
    a.F = m->F;
    a.Fpad = m->Fpad;
    a.act = m->act;
    a.L = m->L;
    const MlpShape sh = (prec == TMD_BF16_MLP) ? pick_act<true>(m->act, m->H, m->L)
                                               : pick_act<false>(m->act, m->H, m->L);
    const int kTileAtoms = sh.waves * 16 * sh.cb;
    int64_t tiles = 0;
    for (int s = 0; s < m->S; ++s) {
        a.sp_off[s] = g.off[s];
        a.tile_off[s] = tiles;
        tiles += (g.off[s + 1] - g.off[s] + kTileAtoms - 1) / kTileAtoms;
    }
    a.sp_off[m->S] = g.off[m->S];
    a.tile_off[m->S] = tiles;
    a.sp_idx = g.idx;
    a.G = G;
    a.Gb = Gb;
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
    const int rlds = resident_lds_bytes(m->H, m->L, m->Fpad);
    ResidentFn rfn = nullptr;
    if (prec == TMD_BF16_MLP && rlds <= kMaxResidentLds && g.off[m->S] >= (int64_t)16 * 16 * ctx->num_cus)
        rfn = m->act == TMD_ACT_SQUAREPLUS ? pick_resident<TMD_ACT_SQUAREPLUS>(m->H, m->L)
                                           : pick_resident<TMD_ACT_TANH>(m->H, m->L);
    if (rfn) {
        TMD_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(rfn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, rlds));
        ProfScope ps_(ctx, "mlp");
        rfn<<<(unsigned)ctx->num_cus, 1024, rlds, ctx->stream>>>(a);
    } else {
        ProfScope ps_(ctx, "mlp");
        sh.fn<<<(unsigned)tiles, sh.waves * 64, 0, ctx->stream>>>(a);
    }
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd
