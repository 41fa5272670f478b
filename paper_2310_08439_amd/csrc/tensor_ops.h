// Per-pair tensor algebra shared by the energy/force kernels and the
// training kernels: the moment monomials M_d(u) in the row order of the
// multiplicity table T_dm (Sec. III.A, eqn T_dm), their adjoint (the F2 term
// of the force, eqn F2_abcx) and their directional derivative (the descriptor
// tangent used by force matching).
#pragma once

#include <hip/hip_runtime.h>

namespace tmd {
namespace ops {

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
    if constexpr (M >= 1) {
        Ax = V[1];
        Ay = V[2];
        Az = V[3];
    }
    if constexpr (M >= 2) {
        Ax += 2.0f * x * V[4] + y * V[5] + z * V[6];
        Ay += x * V[5] + 2.0f * y * V[7] + z * V[8];
        Az += x * V[6] + y * V[8] + 2.0f * z * V[9];
    }
    if constexpr (M >= 3) {
        const float xx = Mv[4], xy = Mv[5], xz = Mv[6], yy = Mv[7], yz = Mv[8], zz = Mv[9];
        Ax += 3.0f * xx * V[10] + 2.0f * xy * V[11] + 2.0f * xz * V[12] + yy * V[13] + yz * V[14] + zz * V[15];
        Ay += xx * V[11] + 2.0f * xy * V[13] + xz * V[14] + 3.0f * yy * V[16] + 2.0f * yz * V[17] + zz * V[18];
        Az += xx * V[12] + xy * V[14] + 2.0f * xz * V[15] + yy * V[17] + 2.0f * yz * V[18] + 3.0f * zz * V[19];
    }
    // sum_d ord(d) V_d M_d = u . A: the monomials of order m are homogeneous of
    // degree m, so u . grad M_d = m M_d (Euler)
    B = x * Ax + y * Ay + z * Az;
}

// Directional derivative of the monomials along t: Mt_d = grad_u M_d . t.
template <int M>
__device__ __forceinline__ void monomial_tangent(const float* Mv, float x, float y, float z, float tx, float ty,
                                                 float tz, float* Mt) {
    Mt[0] = 0.0f;
    if constexpr (M >= 1) {
        Mt[1] = tx;
        Mt[2] = ty;
        Mt[3] = tz;
    }
    if constexpr (M >= 2) {
        Mt[4] = 2.0f * x * tx;
        Mt[5] = tx * y + x * ty;
        Mt[6] = tx * z + x * tz;
        Mt[7] = 2.0f * y * ty;
        Mt[8] = ty * z + y * tz;
        Mt[9] = 2.0f * z * tz;
    }
    if constexpr (M >= 3) {
        const float xx = Mv[4], xy = Mv[5], xz = Mv[6], yy = Mv[7], yz = Mv[8], zz = Mv[9];
        Mt[10] = 3.0f * xx * tx;
        Mt[11] = 2.0f * xy * tx + xx * ty;
        Mt[12] = 2.0f * xz * tx + xx * tz;
        Mt[13] = yy * tx + 2.0f * xy * ty;
        Mt[14] = yz * tx + xz * ty + xy * tz;
        Mt[15] = zz * tx + 2.0f * xz * tz;
        Mt[16] = 3.0f * yy * ty;
        Mt[17] = 2.0f * yz * ty + yy * tz;
        Mt[18] = zz * ty + 2.0f * yz * tz;
        Mt[19] = 3.0f * zz * tz;
    }
}

}  // namespace ops
}  // namespace tmd
